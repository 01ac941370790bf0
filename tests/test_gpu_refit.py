"""Helix refit through the C ABI against the float64 oracle: initial fit
(same discrete decisions, parameters to float32 rounding), chi^2 and the
adjoint gradient (float32 against float64 autograd, and against central
differences), 20 Gauss-Newton steps (parameters within 1e-4 of the float64
fit) and the autograd.Function. Candidates come from the finder on the GPU
side and from the oracle finder on the oracle side (the two are bit-exact,
so candidate c is the same on both)."""
import math

import numpy as np
import pytest

from oracle import OracleConfig, oracle_find_batch
from oracle.refit_oracle import refit_chi2 as o_chi2
from oracle.refit_oracle import refit_gn as o_gn
from oracle.refit_oracle import refit_grad as o_grad
from oracle.refit_oracle import refit_init as o_init
from paper_2511_02742_amd import eventgen

pytestmark = pytest.mark.gpu

# error floors (units of each parameter) below which relative errors are not
# meaningful: kappa [1/mm], phi0 [rad], d0 [mm], z0 [mm], tan_lambda
FLOORS = np.array([1e-4, 1.0, 1.0, 1.0, 0.01])

_cache = {}


def _setup(n_events=48, seed0=1_000_000):
    key = (n_events, seed0)
    if key in _cache:
        return _cache[key]
    import torch
    from paper_2511_02742_amd.hough import HoughFinder, refit_gather
    b = eventgen.poisson_batch(n_events, seed0=seed0)
    dev = torch.device("cuda", 0)
    f = HoughFinder(0)
    t = {k: torch.from_numpy(getattr(b, k)).to(dev) for k in ("r", "z", "vane", "offsets")}
    out = f.find(t["z"], t["vane"], t["offsets"])
    torch.cuda.synchronize()
    hits = refit_gather(out, t["offsets"], t["r"], t["z"], t["vane"])
    # oracle side: its own finder, host gather
    want = oracle_find_batch(OracleConfig(), b.offsets, b.z, b.vane)
    cand = want.cand
    per = []
    for c in cand:
        base = b.offsets[c["event"]]
        idx = base + want.hit_index[c["hit_offset"]:c["hit_offset"] + c["n_hits"]]
        per.append((b.r[idx], b.z[idx], b.vane[idx]))
    _cache[key] = (b, hits, per)
    return _cache[key]


def _rel(a, b):
    return np.abs(a - b) / np.maximum(np.abs(b), FLOORS)


def test_gather_matches_host_gather(gpu_available):
    b, hits, per = _setup()
    off = hits.offsets.cpu().numpy()
    assert len(off) - 1 == len(per)
    r, z, v = hits.r.cpu().numpy(), hits.z.cpu().numpy(), hits.vane.cpu().numpy()
    for c, (rr, zz, vv) in enumerate(per):
        sl = slice(off[c], off[c + 1])
        assert np.array_equal(r[sl], rr) and np.array_equal(z[sl], zz) and np.array_equal(v[sl], vv)


def test_init_matches_oracle(gpu_available):
    from paper_2511_02742_amd.hough import refit_init
    b, hits, per = _setup()
    p = refit_init(hits).cpu().numpy()
    sign, aref, status = hits.sign.cpu().numpy(), hits.aref.cpu().numpy(), hits.status.cpu().numpy()
    off = hits.offsets.cpu().numpy()
    fitted = 0
    for c, (rr, zz, vv) in enumerate(per):
        p0, s0, a0 = o_init(rr, zz, vv)
        # the same candidates are refused (hits on fewer than three vanes, or
        # a line), with status 3
        assert (p0 is None) == (status[c] != 0), (c, status[c])
        if p0 is None:
            assert status[c] == 3
            continue
        fitted += 1
        sl = slice(off[c], off[c + 1])
        assert np.array_equal(sign[sl], s0.astype(np.float32)), c
        assert np.allclose(aref[sl], a0, atol=2e-6), c
        # float64 arithmetic on both sides, then rounded to float32
        assert np.all(_rel(p[c].astype(np.float64), p0) < 2e-6), (c, p[c], p0)
    # the rest are lines of hits on one or two vanes (hits of several tracks
    # stacked at one azimuth), not helices
    assert fitted >= 0.8 * len(per)


def test_chi2_and_adjoint_match_oracle(gpu_available):
    import torch
    from paper_2511_02742_amd.hough import refit_chi2, refit_grad, refit_init
    b, hits, per = _setup()
    p = refit_init(hits)
    # evaluate away from the initial point, where the gradient is not small
    p = p + torch.tensor([0.0, 2e-3, 0.3, 0.4, 5e-3], device=p.device) * torch.ones_like(p)
    p = p.contiguous()
    chi2 = refit_chi2(hits, p).cpu().numpy()
    g = refit_grad(hits, p).cpu().numpy()
    pn = p.cpu().numpy().astype(np.float64)
    sign, aref = hits.sign.cpu().numpy(), hits.aref.cpu().numpy()
    off = hits.offsets.cpu().numpy()
    worst_c = worst_g = 0.0
    status = hits.status.cpu().numpy()
    for c, (rr, zz, vv) in enumerate(per[:120]):
        if status[c] != 0:
            continue
        sl = slice(off[c], off[c + 1])
        wc = o_chi2(pn[c], rr, zz, vv, sign[sl], aref[sl])
        wg = o_grad(pn[c], rr, zz, vv, sign[sl], aref[sl])
        worst_c = max(worst_c, abs(chi2[c] - wc) / max(wc, 1.0))
        # gradient components against the scale of the whole gradient
        worst_g = max(worst_g, float(np.max(np.abs(g[c] * FLOORS - wg * FLOORS)) /
                                     max(np.max(np.abs(wg * FLOORS)), 1e-3)))
    # float32 residuals are good to about 1e-4 sigma; chi^2 here is ~1e3
    assert worst_c < 1e-3, worst_c
    assert worst_g < 1e-3, worst_g


def test_adjoint_matches_central_differences(gpu_available):
    # float32 chi^2 on the GPU, central differences with h = 1e-3 relative
    import torch
    from paper_2511_02742_amd.hough import refit_chi2, refit_grad, refit_init
    b, hits, per = _setup()
    p = refit_init(hits)
    p = (p + torch.tensor([0.0, 2e-3, 0.3, 0.4, 5e-3], device=p.device)).contiguous()
    g = refit_grad(hits, p).double().cpu().numpy()
    fd = np.zeros_like(g)
    for q in range(5):
        h = 1e-3 * p[:, q].abs().clamp(min=1e-3)
        up, dn = p.clone(), p.clone()
        up[:, q] += h
        dn[:, q] -= h
        fd[:, q] = ((refit_chi2(hits, up).double() - refit_chi2(hits, dn).double()) /
                    (up[:, q] - dn[:, q]).double()).cpu().numpy()
    ok = hits.status.cpu().numpy() == 0
    g, fd = g[ok], fd[ok]
    scale = np.maximum(np.abs(g * FLOORS).max(axis=1, keepdims=True), 1e-3)
    err = np.abs((fd - g) * FLOORS) / scale
    # central differences of a float32 chi^2 carry O(h^2) and rounding error
    assert np.median(err) < 1e-3 and np.quantile(err, 0.99) < 5e-2, (np.median(err), err.max())


def _pure(b, c):
    """Whether candidate c (oracle finder) holds hits of one generated track only."""
    want = _oracle_cands(b)
    cd = want.cand[c]
    tr = b.events[cd["event"]].track[want.hit_index[cd["hit_offset"]:cd["hit_offset"] + cd["n_hits"]]]
    return bool(np.all(tr == tr[0]) and tr[0] >= 0)


def _oracle_cands(b):
    key = ("cands", id(b))
    if key not in _cache:
        _cache[key] = oracle_find_batch(OracleConfig(), b.offsets, b.z, b.vane)
    return _cache[key]


def test_gauss_newton_matches_oracle(gpu_available):
    # 20 float32 steps on the GPU against 20 float64 steps of the oracle, each
    # from its own initial fit, on every fitted candidate whose hits all come
    # from one generated track (a helix with a minimum to converge to;
    # candidates mixing tracks have none and both sides wander)
    from paper_2511_02742_amd.hough import refit_gauss_newton, refit_init
    b, hits, per = _setup()
    p = refit_init(hits).contiguous()
    chi2 = refit_gauss_newton(hits, p).cpu().numpy()
    pg = p.cpu().numpy().astype(np.float64)
    status = hits.status.cpu().numpy()
    errs = []
    for c, (rr, zz, vv) in enumerate(per):
        if status[c] != 0 or not _pure(b, c):
            continue
        p0, s0, a0 = o_init(rr, zz, vv)
        po = o_gn(p0, rr, zz, vv, s0, a0)
        e = _rel(pg[c], po)
        e[1] = abs(math.remainder(pg[c][1] - po[1], 2 * math.pi))
        errs.append(e)
        assert np.isfinite(chi2[c])
        if len(errs) == 60:
            break
    errs = np.array(errs)
    assert len(errs) >= 40, len(errs)
    assert np.all(errs.max(axis=0) <= 1e-4), errs.max(axis=0)


def test_autograd_function_backward_is_the_adjoint(gpu_available):
    import torch
    from paper_2511_02742_amd.hough import helix_chi2, refit_grad, refit_init
    b, hits, per = _setup()
    p = refit_init(hits)
    p = (p + torch.tensor([0.0, 1e-3, 0.2, 0.3, 3e-3], device=p.device)).contiguous().requires_grad_(True)
    w = torch.linspace(0.5, 1.5, p.shape[0], device=p.device)
    loss = (w * helix_chi2(p, hits)).sum()
    loss.backward()
    want = refit_grad(hits, p.detach(), w)
    ok = hits.status == 0
    assert torch.allclose(p.grad[ok], want[ok], rtol=1e-6, atol=0.0)


def test_refit_improves_chi2_and_recovers_momentum(gpu_available):
    import torch
    from paper_2511_02742_amd.hough import momentum_mev, refit_chi2, refit_gauss_newton, refit_init
    b, hits, per = _setup()
    p = refit_init(hits).contiguous()
    c0 = refit_chi2(hits, p)
    c1 = refit_gauss_newton(hits, p)
    ok = hits.status == 0
    assert (c1[ok] <= c0[ok] * (1 + 1e-4) + 1e-2).float().mean() > 0.98
    # momentum against the generator truth of the candidate's majority track
    mom = momentum_mev(p.double()).cpu().numpy()
    want = oracle_find_batch(OracleConfig(), b.offsets, b.z, b.vane)
    ratios = []
    status = hits.status.cpu().numpy()
    for c, cd in enumerate(want.cand):
        if status[c] != 0:
            continue
        ev = b.events[cd["event"]]
        tr = ev.track[want.hit_index[cd["hit_offset"]:cd["hit_offset"] + cd["n_hits"]]]
        tr = tr[tr >= 0]
        if len(tr) == 0:
            continue
        t, k = np.unique(tr, return_counts=True)
        if k.max() < cd["n_hits"]:
            continue          # contaminated candidate
        ratios.append(mom[c] / ev.p[t[np.argmax(k)]])
    ratios = np.array(ratios)
    assert len(ratios) > 100
    assert abs(np.median(ratios) - 1.0) < 0.01
    assert np.quantile(np.abs(ratios - 1.0), 0.68) < 0.05
