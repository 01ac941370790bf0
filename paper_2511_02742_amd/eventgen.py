"""Seeded synthetic pileup events for the vane silicon-strip detector.

This module is the input generator shared by the tests, the benchmark and the
CPU oracle's callers. It draws positron helices and records where they cross
the detector vanes; it contains none of the track finder's arithmetic (no
Hough binning, no peak search, no association).

What it stands in for: the paper feeds its finder Geant4/g2esoft RecoHits
(Sec. 3), which are not available here. The geometry follows Sec. 2 and 3:
a 3 T solenoid field along z, muons stored on an orbit of radius about 333 mm
at z = 0, and a detector of 40 radial vanes with silicon strips of 190 um pitch
covering |z| <= 200 mm. Radial acceptance is 90..290 mm (the paper quotes
70..290 mm; the synthetic workload fixes 90 mm).

Event recipe (one numpy PCG64 stream per event, ``default_rng(seed)``):

* per track: start azimuth phi0 ~ U(0, 2pi) on the orbit r0 = 333 mm,
  z0 ~ N(0, 10 mm), |p| ~ U(100, 300) MeV/c, transverse direction
  beta ~ U(0, 2pi), pz/pT ~ U(-0.3, 0.3);
* helix radius R[mm] = pT[MeV/c] / (0.299792458 * B[T]); a positive charge
  turns clockwise seen from +z;
* the helix is followed until r < 90 mm, |z| > 200 mm or 1.5 turns (3 pi of
  turning), whichever comes first;
* a hit is recorded at every crossing of a vane half-plane phi_k = 2 pi k / 40
  with 90 <= r <= 290 mm; r and z are snapped to 0.19 mm strip centres
  (computed in float64, stored float32), the vane id is int16;
* noise: round(noise_frac * n_signal) hits, each on a uniform vane with
  uniform r and z, snapped the same way;
* hits are ordered track by track in arc order, then noise, then shuffled by
  one seeded permutation.

Timeline recipe (time-sliced track finding; ``make_timeline``): muon decays
at times drawn as a Poisson process of a given rate (decays/ns, as the
paper's Table 1 quotes its rates) over a span; each decay emits one positron
drawn as above, whose hit at turning angle a is recorded at time
t_decay + R a sqrt(1 + tan^2 lambda) / c (the positron moves at c, no
timing smearing), stored float32 in ns; noise hits (1 % of the signal) are
uniform in time over the span and in space as above; all hits are sorted by
time (stable: decay order, then arc order, noise last among equal times).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

B_TESLA = 3.0
GEV_PER_T_M = 0.299792458          # pT[MeV/c] = 0.2998 * B[T] * R[mm]
ORBIT_R_MM = 333.0
Z0_SIGMA_MM = 10.0
P_MIN, P_MAX = 100.0, 300.0
TAN_MAX = 0.3                      # |pz/pT|
N_VANES = 40
R_MIN_MM, R_MAX_MM = 90.0, 290.0
Z_MAX_MM = 200.0
PITCH_MM = 0.19
MAX_TURNING = 3.0 * math.pi        # 1.5 turns
C_MM_PER_NS = 299.792458

_N_R_STRIPS = int(math.ceil((R_MAX_MM - R_MIN_MM) / PITCH_MM))
_N_Z_STRIPS = int(math.ceil((2.0 * Z_MAX_MM) / PITCH_MM))


@dataclasses.dataclass
class Event:
    """One pileup event as structure-of-arrays hits plus generator truth."""

    r: np.ndarray          # float32 [n]  radial strip centre, mm
    z: np.ndarray          # float32 [n]  axial strip centre, mm
    vane: np.ndarray       # int16   [n]  vane id in [0, 40)
    track: np.ndarray      # int32   [n]  generating track, -1 for noise
    seed: int
    n_tracks: int
    # per-track truth, length n_tracks
    p: np.ndarray          # |p| MeV/c
    pt: np.ndarray         # transverse momentum MeV/c
    tan_lambda: np.ndarray # pz / pT
    phi0: np.ndarray       # start azimuth on the orbit (rad)
    z0: np.ndarray         # start z (mm)
    beta: np.ndarray       # transverse direction at start (rad)

    @property
    def n_hits(self) -> int:
        return int(self.z.shape[0])


@dataclasses.dataclass
class Batch:
    """Concatenated events with CSR offsets (int64, n_events + 1)."""

    r: np.ndarray
    z: np.ndarray
    vane: np.ndarray
    offsets: np.ndarray
    events: List[Event]

    @property
    def n_events(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def n_hits(self) -> int:
        return int(self.offsets[-1])


def _snap(x: np.ndarray, lo: float, n_strips: int) -> np.ndarray:
    idx = np.floor((x - lo) / PITCH_MM)
    idx = np.clip(idx, 0, n_strips - 1)
    return lo + (idx + 0.5) * PITCH_MM


def _track_crossings(phi0, z0, pt, tanl, beta):
    """Vane crossings of one batch of helices (vectorised over tracks).

    Returns (track_idx, alpha, r, z, vane) for every accepted crossing, in
    no particular order.
    """
    nt = phi0.shape[0]
    radius = pt / (GEV_PER_T_M * B_TESLA)
    p0x = ORBIT_R_MM * np.cos(phi0)
    p0y = ORBIT_R_MM * np.sin(phi0)
    # clockwise motion: the centre lies to the right of the velocity
    cx = p0x + radius * np.sin(beta)
    cy = p0y - radius * np.cos(beta)
    psi0 = beta + 0.5 * math.pi            # angle of (start - centre)

    # turning angle at which |z| leaves the detector
    with np.errstate(divide="ignore", invalid="ignore"):
        a_z = np.where(tanl > 0, (Z_MAX_MM - z0) / (radius * tanl),
                       np.where(tanl < 0, (-Z_MAX_MM - z0) / (radius * tanl), np.inf))
    a_z = np.where(np.abs(z0) > Z_MAX_MM, 0.0, a_z)

    # turning angle at which r first drops below R_MIN:
    # r^2 = |C|^2 + R^2 + 2 R |C| cos(psi - psi_c) < R_MIN^2
    cnorm = np.hypot(cx, cy)
    psic = np.arctan2(cy, cx)
    with np.errstate(divide="ignore", invalid="ignore"):
        kappa = (R_MIN_MM ** 2 - cnorm ** 2 - radius ** 2) / (2.0 * radius * cnorm)
    acos_k = np.arccos(np.clip(kappa, -1.0, 1.0))
    delta0 = np.mod(psi0 - psic, 2.0 * math.pi)
    a_r = np.where(kappa <= -1.0, np.inf,
                   np.mod(delta0 - (2.0 * math.pi - acos_k), 2.0 * math.pi))
    a_stop = np.minimum(np.minimum(a_r, a_z), MAX_TURNING)

    vphi = 2.0 * math.pi * np.arange(N_VANES) / N_VANES
    ux = np.cos(vphi)[None, :]
    uy = np.sin(vphi)[None, :]
    b = ux * cx[:, None] + uy * cy[:, None]                 # [nt, 40]
    disc = b * b - (cnorm ** 2 - radius ** 2)[:, None]
    sq = np.sqrt(np.maximum(disc, 0.0))
    out_t, out_a, out_r, out_z, out_v = [], [], [], [], []
    for sign in (-1.0, 1.0):
        t = b + sign * sq                                    # distance along the vane ray
        ok = (disc >= 0.0) & (t > 0.0)
        px = t * ux
        py = t * uy
        psip = np.arctan2(py - cy[:, None], px - cx[:, None])
        a_base = np.mod(psi0[:, None] - psip, 2.0 * math.pi)
        for turn in (0.0, 2.0 * math.pi):
            a = a_base + turn
            keep = ok & (a < a_stop[:, None]) & (t >= R_MIN_MM) & (t <= R_MAX_MM)
            ti, vi = np.nonzero(keep)
            out_t.append(ti)
            out_a.append(a[ti, vi])
            out_r.append(t[ti, vi])
            out_z.append(z0[ti] + radius[ti] * a[ti, vi] * tanl[ti])
            out_v.append(vi)
    ti = np.concatenate(out_t)
    a = np.concatenate(out_a)
    r = np.concatenate(out_r)
    z = np.concatenate(out_z)
    v = np.concatenate(out_v)
    keep = np.abs(z) <= Z_MAX_MM
    return ti[keep], a[keep], r[keep], z[keep], v[keep]


def make_event(seed: int, n_tracks: int, noise_frac: float = 0.01) -> Event:
    """Generate one event with ``n_tracks`` positrons and uniform noise."""
    rng = np.random.default_rng(seed)
    nt = int(n_tracks)
    phi0 = rng.uniform(0.0, 2.0 * math.pi, nt)
    z0 = rng.normal(0.0, Z0_SIGMA_MM, nt)
    p = rng.uniform(P_MIN, P_MAX, nt)
    beta = rng.uniform(0.0, 2.0 * math.pi, nt)
    tanl = rng.uniform(-TAN_MAX, TAN_MAX, nt)
    pt = p / np.sqrt(1.0 + tanl * tanl)

    if nt > 0:
        ti, a, r, z, v = _track_crossings(phi0, z0, pt, tanl, beta)
        order = np.lexsort((a, ti))              # track order, then arc order
        ti, r, z, v = ti[order], r[order], z[order], v[order]
    else:
        ti = np.zeros(0, np.int64)
        r = z = np.zeros(0)
        v = np.zeros(0, np.int64)
    n_sig = ti.shape[0]
    n_noise = int(math.floor(noise_frac * n_sig + 0.5))
    nv = rng.integers(0, N_VANES, n_noise)
    nr = rng.uniform(R_MIN_MM, R_MAX_MM, n_noise)
    nz = rng.uniform(-Z_MAX_MM, Z_MAX_MM, n_noise)

    r_all = np.concatenate([r, nr])
    z_all = np.concatenate([z, nz])
    v_all = np.concatenate([v, nv])
    t_all = np.concatenate([ti, np.full(n_noise, -1)])
    perm = rng.permutation(r_all.shape[0])
    r_s = _snap(r_all[perm], R_MIN_MM, _N_R_STRIPS).astype(np.float32)
    z_s = _snap(z_all[perm], -Z_MAX_MM, _N_Z_STRIPS).astype(np.float32)
    return Event(r=r_s, z=z_s, vane=v_all[perm].astype(np.int16),
                 track=t_all[perm].astype(np.int32), seed=int(seed), n_tracks=nt,
                 p=p, pt=pt, tan_lambda=tanl, phi0=phi0, z0=z0, beta=beta)


def make_batch(events: Sequence[Event]) -> Batch:
    """Concatenate events into SoA arrays with int64 CSR offsets."""
    counts = np.array([e.n_hits for e in events], dtype=np.int64)
    offsets = np.zeros(len(events) + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    if events:
        r = np.concatenate([e.r for e in events]).astype(np.float32)
        z = np.concatenate([e.z for e in events]).astype(np.float32)
        vane = np.concatenate([e.vane for e in events]).astype(np.int16)
    else:
        r = np.zeros(0, np.float32)
        z = np.zeros(0, np.float32)
        vane = np.zeros(0, np.int16)
    return Batch(r=r, z=z, vane=vane, offsets=offsets, events=list(events))


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

def tiny_event(seed: int = 1) -> Event:
    """1 event, 5 tracks, no noise (the oracle finishes it in well under 1 s)."""
    return make_event(seed, 5, noise_frac=0.0)


def pileup_event(seed: int, n_tracks: int = 50, noise_frac: float = 0.01) -> Event:
    """A heavy-pileup event: ``n_tracks`` positrons plus 1% noise hits."""
    return make_event(seed, n_tracks, noise_frac)


def pileup_batch(n_events: int, n_tracks: int = 50, seed0: int = 0) -> Batch:
    """``n_events`` pileup events with seeds seed0 .. seed0 + n_events - 1."""
    return make_batch([pileup_event(seed0 + i, n_tracks) for i in range(n_events)])


def poisson_batch(n_events: int, mean_tracks: float = 20.0, seed0: int = 1_000_000,
                  lo: int = 1, hi: int = 100) -> Batch:
    """Uneven batch: per-event track count ~ Poisson(mean) clipped to [lo, hi].

    The count is drawn from a stream seeded with the event's seed plus
    2**40, so that it does not consume the event's own stream.
    """
    events = []
    for i in range(n_events):
        s = seed0 + i
        nt = int(np.clip(np.random.default_rng(s + (1 << 40)).poisson(mean_tracks), lo, hi))
        events.append(make_event(s, nt))
    return make_batch(events)


def mixed_pileup_batch(n_events: int, levels: Sequence[int] = (1, 10, 25, 50, 100),
                       seed0: int = 2_000_000) -> Batch:
    """Events whose pileup is drawn uniformly from ``levels``."""
    events = []
    for i in range(n_events):
        s = seed0 + i
        nt = int(levels[int(np.random.default_rng(s + (1 << 40)).integers(0, len(levels)))])
        events.append(make_event(s, nt))
    return make_batch(events)


def hit_histogram(batch: Batch) -> dict:
    n = np.diff(batch.offsets)
    if n.size == 0:
        return {"n_events": 0}
    return {"n_events": int(n.size), "hits_total": int(n.sum()), "hits_min": int(n.min()),
            "hits_mean": float(n.mean()), "hits_max": int(n.max()),
            "hits_p50": float(np.percentile(n, 50)), "hits_p99": float(np.percentile(n, 99))}


# ---------------------------------------------------------------------------
# Timelines: decays spread over time, for the time-sliced finder
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Timeline:
    """Time-ordered hits of muon decays spread over a time span."""

    r: np.ndarray          # float32 [n]
    z: np.ndarray          # float32 [n]
    vane: np.ndarray       # int16   [n]
    t: np.ndarray          # float32 [n]  hit time, ns, non-decreasing
    track: np.ndarray      # int32   [n]  generating decay, -1 for noise
    seed: int
    rate_per_ns: float
    span_ns: float
    t_decay: np.ndarray    # float64 [n_decays]
    p: np.ndarray          # |p| MeV/c per decay

    @property
    def n_hits(self) -> int:
        return int(self.z.shape[0])


@dataclasses.dataclass
class TimelineBatch:
    r: np.ndarray
    z: np.ndarray
    vane: np.ndarray
    t: np.ndarray
    offsets: np.ndarray
    timelines: List[Timeline]

    @property
    def n_timelines(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def n_hits(self) -> int:
        return int(self.offsets[-1])

    def n_windows(self, window_ns: float = 10.0, step_ns: float = 5.0) -> int:
        """Windows [k step, k step + window) that can hold a hit: up to the
        last hit time of any timeline."""
        if self.n_hits == 0:
            return 0
        return int(math.floor(float(self.t.max()) / step_ns)) + 1


def make_timeline(seed: int, rate_per_ns: float, span_ns: float, noise_frac: float = 0.01) -> Timeline:
    """Decays at Poisson times of the given rate over [0, span_ns)."""
    rng = np.random.default_rng(seed)
    nd = int(rng.poisson(rate_per_ns * span_ns))
    t_dec = np.sort(rng.uniform(0.0, span_ns, nd))
    phi0 = rng.uniform(0.0, 2.0 * math.pi, nd)
    z0 = rng.normal(0.0, Z0_SIGMA_MM, nd)
    p = rng.uniform(P_MIN, P_MAX, nd)
    beta = rng.uniform(0.0, 2.0 * math.pi, nd)
    tanl = rng.uniform(-TAN_MAX, TAN_MAX, nd)
    pt = p / np.sqrt(1.0 + tanl * tanl)
    if nd > 0:
        ti, a, r, z, v = _track_crossings(phi0, z0, pt, tanl, beta)
        radius = pt / (GEV_PER_T_M * B_TESLA)
        t = t_dec[ti] + radius[ti] * a * np.sqrt(1.0 + tanl[ti] ** 2) / C_MM_PER_NS
        order = np.lexsort((a, ti))
        ti, r, z, v, t = ti[order], r[order], z[order], v[order], t[order]
    else:
        ti = np.zeros(0, np.int64)
        r = z = t = np.zeros(0)
        v = np.zeros(0, np.int64)
    n_sig = ti.shape[0]
    n_noise = int(math.floor(noise_frac * n_sig + 0.5))
    nv = rng.integers(0, N_VANES, n_noise)
    nr = rng.uniform(R_MIN_MM, R_MAX_MM, n_noise)
    nz = rng.uniform(-Z_MAX_MM, Z_MAX_MM, n_noise)
    nt_ = rng.uniform(0.0, span_ns, n_noise)
    r_all = np.concatenate([r, nr])
    z_all = np.concatenate([z, nz])
    v_all = np.concatenate([v, nv])
    tr_all = np.concatenate([ti, np.full(n_noise, -1)])
    t_all = np.concatenate([t, nt_]).astype(np.float32)
    order = np.argsort(t_all, kind="stable")
    return Timeline(r=_snap(r_all[order], R_MIN_MM, _N_R_STRIPS).astype(np.float32),
                    z=_snap(z_all[order], -Z_MAX_MM, _N_Z_STRIPS).astype(np.float32),
                    vane=v_all[order].astype(np.int16), t=t_all[order], track=tr_all[order].astype(np.int32),
                    seed=int(seed), rate_per_ns=float(rate_per_ns), span_ns=float(span_ns), t_decay=t_dec, p=p)


def make_timeline_batch(timelines: Sequence[Timeline]) -> TimelineBatch:
    counts = np.array([tl.n_hits for tl in timelines], dtype=np.int64)
    offsets = np.zeros(len(timelines) + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    cat = (lambda k, dt: np.concatenate([getattr(tl, k) for tl in timelines]).astype(dt)
           if timelines else np.zeros(0, dt))
    return TimelineBatch(r=cat("r", np.float32), z=cat("z", np.float32), vane=cat("vane", np.int16),
                         t=cat("t", np.float32), offsets=offsets, timelines=list(timelines))


def timeline_batch(n_timelines: int, rate_per_ns: float, span_ns: float, seed0: int = 3_000_000) -> TimelineBatch:
    """``n_timelines`` timelines with seeds seed0 .. seed0 + n - 1."""
    return make_timeline_batch([make_timeline(seed0 + i, rate_per_ns, span_ns) for i in range(n_timelines)])
