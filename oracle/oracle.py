"""ctypes front end of the C oracle (``hough_oracle.c``) -- test infrastructure.

The C file is compiled with ``gcc -O2 -ffp-contract=off`` into
``oracle/liborc_hough.so``; :func:`build_oracle` does it, and the loader
builds it only when no library is present.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hough_oracle.c")
_LIB = os.path.join(_HERE, "liborc_hough.so")

ORC_ERR_DATA = -6

cand_dtype = np.dtype([("event", "<i4"), ("iter", "<i4"), ("theta_bin", "<i4"), ("rho_bin", "<i4"),
                       ("peak_votes", "<u4"), ("n_hits", "<u4"), ("hit_offset", "<i8"),
                       ("theta", "<f4"), ("rho", "<f4")])
assert cand_dtype.itemsize == 40


class _CConfig(ctypes.Structure):
    _fields_ = [("n_theta", ctypes.c_int32), ("n_rho", ctypes.c_int32),
                ("rho_min", ctypes.c_float), ("rho_max", ctypes.c_float),
                ("n_vanes", ctypes.c_int32), ("phi_unit", ctypes.c_int32),
                ("min_votes", ctypes.c_uint32), ("peak_mode", ctypes.c_int32),
                ("nms_radius", ctypes.c_int32), ("assoc_window", ctypes.c_int32),
                ("max_iters", ctypes.c_int32), ("coarse_theta", ctypes.c_int32),
                ("coarse_rho", ctypes.c_int32)]


track_dtype = np.dtype([("timeline", "<i4"), ("track", "<i4"), ("window", "<i4"), ("n_hits", "<i4"),
                        ("hit_offset", "<i8"), ("vane_first", "<i4"), ("vane_last", "<i4"),
                        ("theta_bin", "<i4"), ("rho_bin", "<i4"), ("last_window", "<i4"), ("carried", "<i4")])
assert track_dtype.itemsize == 48


class _CTwConfig(ctypes.Structure):
    _fields_ = [("window_ns", ctypes.c_float), ("step_ns", ctypes.c_float), ("gate_r", ctypes.c_float),
                ("gate_z", ctypes.c_float), ("gate_t", ctypes.c_float), ("max_track_hits", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 2)]


@dataclasses.dataclass
class TwConfig:
    """Time windows and track extension (window width and step in ns, the
    extrapolation gates in mm and ns, the longest track)."""
    window_ns: float = 10.0
    step_ns: float = 5.0
    gate_r: float = 10.0
    gate_z: float = 4.0
    gate_t: float = 2.0
    max_track_hits: int = 64

    def c(self) -> _CTwConfig:
        return _CTwConfig(self.window_ns, self.step_ns, self.gate_r, self.gate_z, self.gate_t,
                          self.max_track_hits)


@dataclasses.dataclass
class OracleConfig:
    n_theta: int = 1024
    n_rho: int = 1024
    rho_min: float = -500.0
    rho_max: float = 500.0
    n_vanes: int = 40
    phi_unit: int = 0          # 0 degrees, 1 radians
    min_votes: int = 6
    peak_mode: int = 1         # 0 argmax, 1 nms, 2 coarse-to-fine
    nms_radius: int = 1
    assoc_window: int = 0
    max_iters: int = 0
    coarse_theta: int = 10     # peak_mode 2: fine bins per coarse bin
    coarse_rho: int = 10

    def c(self) -> _CConfig:
        return _CConfig(self.n_theta, self.n_rho, self.rho_min, self.rho_max, self.n_vanes,
                        self.phi_unit, self.min_votes, self.peak_mode, self.nms_radius,
                        self.assoc_window, self.max_iters, self.coarse_theta, self.coarse_rho)


def build_oracle(force: bool = True) -> str:
    """Compile the oracle shared library (always when ``force``)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
                               "-Wall", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build_oracle(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        cfgp = ctypes.POINTER(_CConfig)
        lib.orc_tables.argtypes = [cfgp, P, P, P, P, P, P]
        lib.orc_tables.restype = ctypes.c_int
        lib.orc_bin_index.argtypes = [cfgp, ctypes.c_float, ctypes.c_float, ctypes.c_int32]
        lib.orc_bin_index.restype = ctypes.c_int32
        lib.orc_fill.argtypes = [cfgp, I64, P, P, P, P]
        lib.orc_fill.restype = I64
        lib.orc_peaks.argtypes = [cfgp, P, P, I64]
        lib.orc_peaks.restype = I64
        lib.orc_find.argtypes = [cfgp, ctypes.c_int32, I64, P, P, P, I64, P, I64, P, P]
        lib.orc_find.restype = ctypes.c_int
        lib.orc_acc_after.argtypes = [cfgp, I64, P, P, ctypes.c_int32, P]
        lib.orc_acc_after.restype = ctypes.c_int
        lib.orc_find_batch.argtypes = [cfgp, ctypes.c_int32, P, P, P, P, I64, P, I64, P]
        lib.orc_find_batch.restype = ctypes.c_int
        twp = ctypes.POINTER(_CTwConfig)
        lib.orc_tw_find_batch.argtypes = [cfgp, twp, ctypes.c_int32, P, P, P, P, P, ctypes.c_int32, P, I64, P,
                                          I64, P]
        lib.orc_tw_find_batch.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _hits(z, vane):
    z = np.ascontiguousarray(z, dtype=np.float32)
    vane = np.ascontiguousarray(vane, dtype=np.int16)
    if z.shape != vane.shape:
        raise ValueError("z and vane must have the same length")
    return z, vane


class OracleError(RuntimeError):
    def __init__(self, status: int):
        super().__init__("oracle status %d" % status)
        self.status = status


def oracle_tables(cfg: OracleConfig):
    """(cos_t, sin_t, phi_v, inv_w, theta_c, rho_c) as float32 arrays."""
    lib = _load()
    c = cfg.c()
    cos_t = np.empty(cfg.n_theta, np.float32)
    sin_t = np.empty(cfg.n_theta, np.float32)
    theta_c = np.empty(cfg.n_theta, np.float32)
    phi_v = np.empty(cfg.n_vanes, np.float32)
    rho_c = np.empty(cfg.n_rho, np.float32)
    inv_w = np.empty(1, np.float32)
    st = lib.orc_tables(ctypes.byref(c), _ptr(cos_t), _ptr(sin_t), _ptr(phi_v), _ptr(inv_w),
                        _ptr(theta_c), _ptr(rho_c))
    if st:
        raise OracleError(st)
    return cos_t, sin_t, phi_v, inv_w[0], theta_c, rho_c


def oracle_bin(cfg: OracleConfig, phi: float, z: float, j: int) -> int:
    """Raw (unclipped) rho bin of a hit at theta row j."""
    c = cfg.c()
    return int(_load().orc_bin_index(ctypes.byref(c), ctypes.c_float(phi), ctypes.c_float(z), j))


def oracle_fill(cfg: OracleConfig, z, vane, alive=None):
    """Accumulator (uint32 [n_theta, n_rho]) and the number of dropped votes."""
    z, vane = _hits(z, vane)
    c = cfg.c()
    acc = np.empty((cfg.n_theta, cfg.n_rho), np.uint32)
    al = None
    if alive is not None:
        al = np.ascontiguousarray(alive, dtype=np.uint8)
    r = _load().orc_fill(ctypes.byref(c), z.shape[0], _ptr(z), _ptr(vane),
                         _ptr(al) if al is not None else None, _ptr(acc))
    if r < 0:
        raise OracleError(int(r))
    return acc, int(r)


def oracle_peaks(cfg: OracleConfig, acc: np.ndarray, cap: int = 1 << 20) -> np.ndarray:
    """Peak keys (uint64, descending) of a given accumulator."""
    acc = np.ascontiguousarray(acc, dtype=np.uint32)
    assert acc.shape == (cfg.n_theta, cfg.n_rho)
    c = cfg.c()
    keys = np.empty(cap, np.uint64)
    n = _load().orc_peaks(ctypes.byref(c), _ptr(acc), _ptr(keys), cap)
    if n < 0:
        raise OracleError(int(n))
    return keys[:min(n, cap)].copy()


@dataclasses.dataclass
class FindResult:
    cand: np.ndarray        # structured, cand_dtype
    hit_index: np.ndarray   # int32
    claim: np.ndarray       # int32 per hit (single-event form only)
    n_iters: int
    votes: int


def oracle_find(cfg: OracleConfig, z, vane, event_id: int = 0) -> FindResult:
    z, vane = _hits(z, vane)
    n = z.shape[0]
    cap = n // cfg.min_votes + 1
    cand = np.zeros(cap, cand_dtype)
    hits = np.zeros(max(n, 1), np.int32)
    claim = np.zeros(max(n, 1), np.int32)
    out = np.zeros(4, np.int64)
    c = cfg.c()
    st = _load().orc_find(ctypes.byref(c), event_id, n, _ptr(z), _ptr(vane), _ptr(cand), cap,
                          _ptr(hits), n, _ptr(claim), _ptr(out))
    if st:
        raise OracleError(st)
    return FindResult(cand[:out[0]].copy(), hits[:out[1]].copy(), claim[:n].copy(),
                      int(out[2]), int(out[3]))


def oracle_find_batch(cfg: OracleConfig, offsets, z, vane) -> FindResult:
    z, vane = _hits(z, vane)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    ne = offsets.shape[0] - 1
    n = int(offsets[-1]) if ne >= 0 and offsets.shape[0] else 0
    cap = n // cfg.min_votes + 1
    cand = np.zeros(cap, cand_dtype)
    hits = np.zeros(max(n, 1), np.int32)
    out = np.zeros(4, np.int64)
    c = cfg.c()
    st = _load().orc_find_batch(ctypes.byref(c), ne, _ptr(offsets), _ptr(z), _ptr(vane),
                                _ptr(cand), cap, _ptr(hits), n, _ptr(out))
    if st:
        raise OracleError(st)
    return FindResult(cand[:out[0]].copy(), hits[:out[1]].copy(), np.zeros(0, np.int32),
                      int(out[2]), int(out[3]))


def oracle_acc_after(cfg: OracleConfig, z, vane, iters: int) -> np.ndarray:
    z, vane = _hits(z, vane)
    acc = np.empty((cfg.n_theta, cfg.n_rho), np.uint32)
    c = cfg.c()
    st = _load().orc_acc_after(ctypes.byref(c), z.shape[0], _ptr(z), _ptr(vane), iters, _ptr(acc))
    if st:
        raise OracleError(st)
    return acc


def _batch_slice(job):
    cfg, offsets, z, vane = job
    r = oracle_find_batch(cfg, offsets, z, vane)
    return r.cand, r.hit_index, r.n_iters, r.votes


def oracle_find_batch_sliced(cfg: OracleConfig, offsets, z, vane, workers: int = 16) -> FindResult:
    """oracle_find_batch over contiguous event slices in independent worker
    processes, concatenated: the same arrays as one oracle_find_batch call
    (events are independent), only sooner. Each worker runs the unchanged
    single-threaded oracle."""
    import multiprocessing as mp
    z, vane = _hits(z, vane)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    ne = offsets.shape[0] - 1
    workers = max(1, min(int(workers), ne))
    if workers == 1:
        return oracle_find_batch(cfg, offsets, z, vane)
    bounds = np.linspace(0, ne, workers + 1).astype(np.int64)
    jobs = []
    for w in range(workers):
        e0, e1 = int(bounds[w]), int(bounds[w + 1])
        lo, hi = int(offsets[e0]), int(offsets[e1])
        jobs.append((cfg, offsets[e0:e1 + 1] - lo, z[lo:hi].copy(), vane[lo:hi].copy()))
    with mp.get_context("spawn").Pool(workers) as pool:
        parts = pool.map(_batch_slice, jobs)
    cands, hits = [], []
    hbase = 0
    n_iters = votes = 0
    for w, (c, h, it, vt) in enumerate(parts):
        c = c.copy()
        c["event"] += int(bounds[w])
        c["hit_offset"] += hbase
        hbase += len(h)
        cands.append(c)
        hits.append(h)
        n_iters = max(n_iters, it)     # a batch reports its largest iteration count
        votes += vt
    return FindResult(np.concatenate(cands), np.concatenate(hits).astype(np.int32), np.zeros(0, np.int32),
                      n_iters, votes)


@dataclasses.dataclass
class TrackResult:
    tracks: np.ndarray      # structured, track_dtype
    hit_index: np.ndarray   # int32, timeline-local, vane order from each track's lower end
    n_candidates: int       # Hough candidates over all windows
    n_carried: int          # track-windows in which a flagged track gained hits


def oracle_tw_find_batch(cfg: OracleConfig, tw: TwConfig, offsets, r, z, vane, t, n_windows: int) -> TrackResult:
    """Time-sliced track finding with track extension over CSR timelines."""
    z, vane = _hits(z, vane)
    r = np.ascontiguousarray(r, dtype=np.float32)
    t = np.ascontiguousarray(t, dtype=np.float32)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    n_tl = offsets.shape[0] - 1
    n = int(offsets[-1]) if offsets.shape[0] else 0
    kcap = n // 3 + n_tl + 1
    tracks = np.zeros(kcap, track_dtype)
    hits = np.zeros(max(n, 1), np.int32)
    out = np.zeros(4, np.int64)
    c, w = cfg.c(), tw.c()
    st = _load().orc_tw_find_batch(ctypes.byref(c), ctypes.byref(w), n_tl, _ptr(offsets), _ptr(r), _ptr(z),
                                   _ptr(vane), _ptr(t), int(n_windows), _ptr(tracks), kcap, _ptr(hits),
                                   max(n, 1), _ptr(out))
    if st:
        raise OracleError(st)
    return TrackResult(tracks[:out[0]].copy(), hits[:out[1]].copy(), int(out[2]), int(out[3]))
