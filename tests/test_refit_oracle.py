"""Pins of the float64 refit oracle (no GPU). The exact hits used here are found
by marching along a known helix and bisecting each vane-plane crossing, not by
the analytic circle-ray root the residuals use."""
import math

import numpy as np
import pytest

from oracle.refit_oracle import (GN_STEPS, SIGMA_MM, momentum_mev, refit_chi2, refit_gn, refit_grad, refit_init,
                                 refit_residuals, truth_params)

pytestmark = pytest.mark.filterwarnings("ignore::UserWarning")


def helix_hits(p, a_lo, a_hi, n_vanes=40, step=2e-4, r_lo=90.0, r_hi=290.0):
    """Exact (r, z, vane, a) of every crossing of the helix p with a vane
    half-plane for turning angles in [a_lo, a_hi], by dense marching and
    bisection on the turning angle."""
    kappa, phi0, d0, z0, tl = p
    R = 1.0 / kappa
    n = np.array([math.sin(phi0), -math.cos(phi0)])
    c = (d0 + R) * n
    psi0 = math.atan2(-n[1], -n[0])            # angle of (perigee - centre)

    def pos(a):
        return c + R * np.array([math.cos(psi0 - a), math.sin(psi0 - a)])

    out = []
    a_grid = np.arange(a_lo, a_hi, step)
    P = c[:, None] + R * np.stack([np.cos(psi0 - a_grid), np.sin(psi0 - a_grid)])
    for k in range(n_vanes):
        ph = 2 * math.pi * k / n_vanes
        u = np.array([math.cos(ph), math.sin(ph)])
        f = u[0] * P[1] - u[1] * P[0]
        front = u[0] * P[0] + u[1] * P[1] > 0
        idx = np.nonzero((np.sign(f[:-1]) != np.sign(f[1:])) & front[:-1] & front[1:])[0]
        for i in idx:
            lo, hi = a_grid[i], a_grid[i + 1]
            flo = u[0] * pos(lo)[1] - u[1] * pos(lo)[0]
            for _ in range(80):
                mid = 0.5 * (lo + hi)
                q = pos(mid)
                fm = u[0] * q[1] - u[1] * q[0]
                if (fm < 0) == (flo < 0):
                    lo, flo = mid, fm
                else:
                    hi = mid
            a = 0.5 * (lo + hi)
            q = pos(a)
            r = math.hypot(q[0], q[1])
            if r_lo <= r <= r_hi:
                out.append((r, z0 + R * a * tl, k, a))
    out.sort(key=lambda h: h[3])
    h = np.array(out)
    return h[:, 0], h[:, 1], h[:, 2].astype(np.int16), h[:, 3]


# a positron leaving the storage orbit inwards: pT = 200 MeV/c, pz/pT = 0.12;
# its circle crosses the detector in one arc through 11 vane planes (one of
# them twice), turning angles -0.87 .. 0.41 rad around the perigee
TRUTH = truth_params(phi_start=0.7, z_start=3.0, pt=200.0, tan_lambda=0.12, beta=0.7 + math.pi + 0.4)


def _track(p=TRUTH):
    r, z, v, a = helix_hits(p, -math.pi + 0.01, math.pi - 0.01)
    assert len(r) >= 8
    return r, z, v, a


def test_exact_hits_lie_on_the_helix():
    r, z, v, a = _track()
    assert len(r) == 11 and len(set(v.tolist())) == 10
    assert np.all((r >= 90) & (r <= 290))
    # each hit is on its vane's ray and on the circle
    kappa, phi0, d0, z0, tl = TRUTH
    c = (d0 + 1 / kappa) * np.array([math.sin(phi0), -math.cos(phi0)])
    ph = 2 * math.pi * v / 40
    x, y = r * np.cos(ph), r * np.sin(ph)
    assert np.allclose(np.hypot(x - c[0], y - c[1]), 1 / kappa, atol=1e-8)


def test_init_recovers_an_exact_helix():
    r, z, v, a = _track()
    p0, sign, aref = refit_init(r, z, v)
    assert np.allclose(p0, TRUTH, rtol=1e-9, atol=1e-9), (p0, TRUTH)
    # the unwrapped turning angles are the true ones
    assert np.allclose(aref, a, atol=1e-9)


def test_chi2_and_gradient_vanish_at_truth():
    r, z, v, a = _track()
    _, sign, aref = refit_init(r, z, v)
    assert refit_chi2(TRUTH, r, z, v, sign, aref) < 1e-14
    # the truth is a fixed point of the fit: a Gauss-Newton step from it (the
    # gradient scaled by the curvature) does not move it
    p1 = refit_gn(TRUTH, r, z, v, sign, aref, steps=1)
    assert np.allclose(p1, TRUTH, rtol=1e-10, atol=1e-12), p1 - TRUTH


def test_residual_scale_is_sigma():
    # moving z0 by one sigma moves every z residual by exactly -1
    r, z, v, a = _track()
    _, sign, aref = refit_init(r, z, v)
    p = TRUTH.copy()
    p[3] += SIGMA_MM
    e = refit_residuals(p, r, z, v, sign, aref).numpy()
    n = len(r)
    assert np.allclose(e[:n], 0.0, atol=1e-9) and np.allclose(e[n:], -1.0, atol=1e-9)
    assert abs(refit_chi2(p, r, z, v, sign, aref) - n) < 1e-8


def test_gradient_matches_central_differences():
    r, z, v, a = _track()
    _, sign, aref = refit_init(r, z, v)
    p = TRUTH * np.array([1.01, 1.0, 1.0, 1.0, 1.0]) + np.array([0.0, 0.004, 0.3, 0.5, 0.01])
    g = refit_grad(p, r, z, v, sign, aref)
    for i in range(5):
        h = 1e-6 * max(abs(p[i]), 1e-3)
        up, dn = p.copy(), p.copy()
        up[i] += h
        dn[i] -= h
        fd = (refit_chi2(up, r, z, v, sign, aref) - refit_chi2(dn, r, z, v, sign, aref)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(g[i]), 1.0), (i, fd, g[i])


def test_gauss_newton_converges_to_truth_from_a_displaced_start():
    r, z, v, a = _track()
    _, sign, aref = refit_init(r, z, v)
    p_start = TRUTH * np.array([1.03, 1.0, 1.0, 1.0, 1.0]) + np.array([0.0, 0.01, 0.8, 1.5, 0.02])
    p = refit_gn(p_start, r, z, v, sign, aref, steps=GN_STEPS)
    assert np.allclose(p, TRUTH, rtol=1e-8, atol=1e-8), (p, TRUTH)


def test_rotation_by_one_vane():
    # rotating the detector by one vane rotates phi0 by 2 pi / 40 and leaves
    # everything else, and the chi^2, unchanged
    r, z, v, a = _track()
    p0, sign, aref = refit_init(r, z, v)
    q = TRUTH.copy()
    q[1] += 2 * math.pi / 40
    v2 = ((v.astype(np.int32) + 1) % 40).astype(np.int16)
    r2, z2, w2, a2 = helix_hits(q, -math.pi + 0.01, math.pi - 0.01)
    assert np.allclose(np.sort(r2), np.sort(r), atol=1e-9)
    q0, sign2, aref2 = refit_init(r, z, v2)
    d = (q0 - p0)
    assert abs(math.remainder(d[1], 2 * math.pi) - 2 * math.pi / 40) < 1e-9
    assert np.allclose(np.delete(q0, 1), np.delete(p0, 1), rtol=1e-9, atol=1e-9)
    p = TRUTH * np.array([1.01, 1, 1, 1, 1]) + np.array([0, 0.003, 0.2, 0.3, 0.004])
    p2 = p.copy()
    p2[1] += 2 * math.pi / 40
    assert abs(refit_chi2(p, r, z, v, sign, aref) - refit_chi2(p2, r, z, v2, sign2, aref2)) < 1e-8


def test_momentum_of_the_truth_parameters():
    pt = 180.0
    q = truth_params(phi_start=2.0, z_start=-4.0, pt=pt, tan_lambda=-0.2, beta=1.1)
    assert abs(momentum_mev(q) - pt * math.sqrt(1 + 0.04)) < 1e-9


def test_generator_track_refit_is_physical():
    # snapped hits of a generated positron: the fit lands near the truth
    from paper_2511_02742_amd import eventgen
    ev = eventgen.make_event(31, 6, noise_frac=0.0)
    done = 0
    for t in range(ev.n_tracks):
        sel = ev.track == t
        if sel.sum() < 6:
            continue
        r, z, v = ev.r[sel], ev.z[sel], ev.vane[sel]
        p0, sign, aref = refit_init(r, z, v)
        p = refit_gn(p0, r, z, v, sign, aref)
        e = refit_residuals(p, r, z, v, sign, aref).numpy()
        assert np.sqrt(np.mean(e ** 2)) < 3.0            # residuals of a few sigma at most
        assert abs(momentum_mev(p) / ev.p[t] - 1.0) < 0.05
        done += 1
    assert done >= 2


# --- refusal rule (a reading: the paper is silent on which candidates a helix
# fit should skip) and the flat-track branch of the turning-angle unwrap ---

def _vane_circle_hits(cx, cy, R, vanes, n_vanes=40):
    """Exact crossings (r, vane) of the circle (centre (cx, cy), radius R) with
    the given vane rays: the root of |t u - c|^2 = R^2 nearest the origin
    that lies in front of it."""
    rs, vs = [], []
    for k in vanes:
        ph = 2 * math.pi * k / n_vanes
        b = math.cos(ph) * cx + math.sin(ph) * cy
        disc = b * b - (cx * cx + cy * cy - R * R)
        assert disc > 0
        t = b - math.sqrt(disc)
        assert t > 0
        rs.append(t)
        vs.append(k)
    return np.array(rs), np.array(vs, np.int16)


def test_two_vanes_are_refused_three_are_fitted():
    r, z, v, a = _track()
    # the truth track crosses one vane plane twice; that pair plus one hit on
    # a second vane is three hits on two vanes: refused
    vals, cnt = np.unique(v, return_counts=True)
    twice = vals[cnt == 2][0]
    pair = np.nonzero(v == twice)[0]
    other = np.nonzero(v != twice)[0][0]
    sel = np.concatenate([pair, [other]])
    p0, _, _ = refit_init(r[sel], z[sel], v[sel])
    assert p0 is None
    # three hits on three distinct vanes define the circle and the z line
    # exactly: the initial fit returns the truth
    sel3 = np.concatenate([pair[:1], np.nonzero(v != twice)[0][[0, 3]]])
    assert len(set(v[sel3].tolist())) == 3
    p0, _, aref = refit_init(r[sel3], z[sel3], v[sel3])
    assert p0 is not None
    assert np.allclose(p0, TRUTH, rtol=1e-9, atol=1e-9), (p0, TRUTH)
    assert np.allclose(aref, a[sel3], atol=1e-9)
    # two hits are refused whatever their vanes
    assert refit_init(r[sel3[:2]], z[sel3[:2]], v[sel3[:2]])[0] is None


def test_straight_lines_are_refused():
    # hits on the straight line x = 150 mm (vanes at -9, 0, 9 and 18 degrees)
    vanes = np.array([39, 0, 1, 2], np.int16)
    ph = 2 * math.pi * vanes / 40
    r = 150.0 / np.cos(ph)
    z = np.array([1.0, 2.0, 3.0, 4.0])
    assert refit_init(r, z, vanes)[0] is None
    # exact circles through the detector: radius 2e4 mm is above the 1e4 mm
    # limit (refused), radius 5e3 mm is below it (fitted, radius recovered)
    for R, fitted in ((2.0e4, False), (5.0e3, True)):
        d0 = 150.0
        cx, cy = d0 + R, 0.0
        r, v = _vane_circle_hits(cx, cy, R, [37, 38, 39, 0, 1, 2, 3])
        z = 0.2 * np.arange(len(r))
        p0, _, _ = refit_init(r, z, v)
        if not fitted:
            assert p0 is None
        else:
            assert p0 is not None
            assert abs(1.0 / p0[0] - R) < 1e-6 * R and abs(p0[2] - d0) < 1e-6


@pytest.mark.parametrize("tan_lambda", [0.0, 0.0015])
def test_flat_track_unwraps_between_the_sides_of_the_largest_gap(tan_lambda):
    # a z spread under 1 mm takes the largest-gap branch: the arc through the
    # detector is contiguous, so the largest angular gap is the rest of the
    # circle and the unwrapped angles are the true turning angles
    truth = TRUTH.copy()
    truth[4] = tan_lambda
    r, z, v, a = helix_hits(truth, -math.pi + 0.01, math.pi - 0.01)
    assert len(r) == 11 and np.ptp(z) < 1.0
    p0, _, aref = refit_init(r, z, v)
    assert np.allclose(aref, a, atol=1e-9)
    assert np.allclose(p0, truth, rtol=1e-9, atol=1e-9), (p0, truth)
    # the same hits in another order unwrap the same way
    perm = np.random.default_rng(5).permutation(len(r))
    p1, _, aref1 = refit_init(r[perm], z[perm], v[perm])
    assert np.allclose(aref1, a[perm], atol=1e-9) and np.allclose(p1, p0, rtol=1e-9, atol=1e-12)


def test_full_circle_flat_track_starts_after_the_largest_gap():
    # a circle wholly inside the detector (perigee 100 mm, apogee 220 mm) with
    # tan lambda = 0: every unwrapped angle is its true angle modulo 2 pi, the
    # span is under one turn, and it starts at the hit that follows the
    # largest gap between neighbouring angles
    R = 60.0
    truth = np.array([1.0 / R, 0.3, 100.0, -5.0, 0.0])
    r, z, v, a = helix_hits(truth, -math.pi + 1e-3, math.pi - 1e-3)
    p0, _, aref = refit_init(r, z, v)
    assert np.allclose(p0[[0, 2, 3, 4]], truth[[0, 2, 3, 4]], rtol=1e-9, atol=1e-9)
    assert abs(math.remainder(p0[1] - truth[1], 2 * math.pi)) < 1e-9
    d = np.mod(aref - a, 2 * math.pi)
    assert np.all(np.minimum(d, 2 * math.pi - d) < 1e-9)
    assert np.ptp(aref) < 2 * math.pi
    srt = np.sort(a)
    gaps = np.append(np.diff(srt), srt[0] + 2 * math.pi - srt[-1])
    start = srt[(int(np.argmax(gaps)) + 1) % len(srt)]
    assert abs(aref.min() - start) < 1e-9
