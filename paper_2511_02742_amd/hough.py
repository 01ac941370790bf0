"""Python binding of ``libhough_tf.so`` (the C ABI in include/hough_tf.h).

Argument marshalling only: torch provides device memory and the stream, and
every step of the finder runs in the library's HIP kernels. There is no CPU
fallback -- if the library is missing the import fails.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhough_tf.so")

HOUGH_OK = 0
HOUGH_ERR_INVALID_ARG = -1
HOUGH_ERR_CAPACITY = -2
HOUGH_ERR_OOM = -3
HOUGH_ERR_DEVICE = -4
HOUGH_ERR_INTERNAL = -5
HOUGH_ERR_DATA = -6

HOUGH_COUNTS = 16
HOUGH_NOALLOC_SCRATCH_BYTES = 64 << 20   # device scratch of hough_find_noalloc
COUNT_NAMES = ("candidates", "hits", "status", "detail", "evals", "iters", "max_iters", "passes",
               "tiled", "truncations", "hot_scans", "hotset_full", "recounts", "large", "votes", "ordered")

EXPORTS = ("hough_config_default", "hough_create", "hough_destroy", "hough_output_bounds", "hough_find", "hough_find_noalloc",
           "hough_tw_config_default", "hough_tw_find",
           "hough_debug_accumulator", "hough_tables", "hough_launch_shape", "hough_set_timing",
           "hough_timing", "hough_set_event_clock", "hough_clock_rate", "hough_graph_create", "hough_graph_launch", "hough_graph_destroy",
           "hough_autotune", "hough_server_create", "hough_server_destroy", "hough_server_clock",
           "hough_server_submit", "hough_server_poll", "hough_server_drain", "hough_server_get_stats",
           "hough_refit_gather", "hough_refit_init", "hough_refit_chi2", "hough_refit_grad",
           "hough_refit_gauss_newton", "hough_lds_peak", "hough_status_string", "hough_last_error")

cand_dtype = np.dtype([("event", "<i4"), ("iter", "<i4"), ("theta_bin", "<i4"), ("rho_bin", "<i4"),
                       ("peak_votes", "<u4"), ("n_hits", "<u4"), ("hit_offset", "<i8"),
                       ("theta", "<f4"), ("rho", "<f4")])
assert cand_dtype.itemsize == 40


class HoughConfig(ctypes.Structure):
    _fields_ = [("n_theta", ctypes.c_int32), ("n_rho", ctypes.c_int32),
                ("rho_min", ctypes.c_float), ("rho_max", ctypes.c_float),
                ("n_vanes", ctypes.c_int32), ("phi_unit", ctypes.c_int32),
                ("min_votes", ctypes.c_uint32), ("peak_mode", ctypes.c_int32),
                ("nms_radius", ctypes.c_int32), ("assoc_window", ctypes.c_int32),
                ("max_iters", ctypes.c_int32), ("tile_rows", ctypes.c_int32),
                ("wg_threads", ctypes.c_int32), ("sweep_groups", ctypes.c_int32),
                ("sweep_threads", ctypes.c_int32), ("coarse_theta", ctypes.c_int32),
                ("coarse_rho", ctypes.c_int32)]


class TwConfig(ctypes.Structure):
    """hough_tw_config: time windows and track extension."""
    _fields_ = [("window_ns", ctypes.c_float), ("step_ns", ctypes.c_float), ("gate_r_mm", ctypes.c_float),
                ("gate_z_mm", ctypes.c_float), ("gate_t_ns", ctypes.c_float), ("max_track_hits", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 2)]


track_dtype = np.dtype([("timeline", "<i4"), ("track", "<i4"), ("window", "<i4"), ("n_hits", "<i4"),
                        ("hit_offset", "<i8"), ("vane_first", "<i4"), ("vane_last", "<i4"),
                        ("theta_bin", "<i4"), ("rho_bin", "<i4"), ("last_window", "<i4"), ("carried", "<i4")])
assert track_dtype.itemsize == 48
TW_COUNT_NAMES = ("tracks", "hits", "status", "detail", "windows", "candidates", "continued")


def tw_config(**overrides) -> TwConfig:
    """The library's default time-window configuration with overrides."""
    lib = load_library()
    tw = TwConfig()
    st = lib.hough_tw_config_default(ctypes.byref(tw))
    if st != HOUGH_OK:
        raise HoughError(st, "hough_tw_config_default")
    for k, v in overrides.items():
        setattr(tw, k, v)
    return tw


class ServerConfig(ctypes.Structure):
    _fields_ = [("lanes", ctypes.c_int32), ("max_batch_events", ctypes.c_int32),
                ("max_batch_hits", ctypes.c_int64), ("queue_hits", ctypes.c_int64),
                ("queue_events", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("device_bytes", ctypes.c_int64)]


served_dtype = np.dtype([("tag", "<u8"), ("status", "<i4"), ("n_hits", "<i4"), ("n_candidates", "<i4"),
                         ("lane", "<i4"), ("cand_offset", "<i8"), ("hit_offset", "<i8"),
                         ("n_hit_index", "<i8"), ("t_arrival", "<f8"), ("t_admit", "<f8"),
                         ("t_done", "<f8")])
assert served_dtype.itemsize == 72

SERVER_STAT_NAMES = ("submitted", "refused", "completed", "launches", "launched_events", "launched_hits",
                     "pending_events", "max_pending_events", "max_lanes_busy", "device_bytes",
                     "results_waiting", "device_bytes_in_use", "max_device_bytes_in_use")


class HoughError(RuntimeError):
    def __init__(self, status: int, detail: str = ""):
        self.status = status
        super().__init__("hough status %d (%s)%s" % (status, _status_string(status),
                                                     (": " + detail) if detail else ""))


_lib = None


def load_library(path: str = LIB_PATH):
    """Loads the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libhough_tf.so not found at %s; run __graft_entry__.build() "
                          "(python -c 'import __graft_entry__ as g; g.build()')" % path)
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    I32 = ctypes.c_int32
    I64 = ctypes.c_int64
    cfgp = ctypes.POINTER(HoughConfig)
    st = ctypes.c_int
    lib.hough_config_default.argtypes = [cfgp]
    lib.hough_config_default.restype = st
    lib.hough_create.argtypes = [cfgp, ctypes.c_int, ctypes.POINTER(P)]
    lib.hough_create.restype = st
    lib.hough_destroy.argtypes = [P]
    lib.hough_destroy.restype = st
    lib.hough_output_bounds.argtypes = [P, I32, I64, ctypes.POINTER(I64), ctypes.POINTER(I64)]
    lib.hough_output_bounds.restype = st
    lib.hough_find.argtypes = [P, P, I32, I64, P, P, P, P, I64, P, I64, P]
    lib.hough_find.restype = st
    lib.hough_find_noalloc.argtypes = [P, P, I32, I64, P, P, P, P, I64, P, I64, P]
    lib.hough_find_noalloc.restype = st
    lib.hough_tw_config_default.argtypes = [P]
    lib.hough_tw_config_default.restype = st
    lib.hough_tw_find.argtypes = [P, P, P, I32, I64, P, P, P, P, P, I32, P, I64, P, I64, P]
    lib.hough_tw_find.restype = st
    lib.hough_debug_accumulator.argtypes = [P, P, I64, P, P, I32, P, P]
    lib.hough_debug_accumulator.restype = st
    lib.hough_tables.argtypes = [P, P, P, P, P, P, P]
    lib.hough_tables.restype = st
    lib.hough_launch_shape.argtypes = [P, ctypes.POINTER(I32), ctypes.POINTER(I32), ctypes.POINTER(I32)]
    lib.hough_launch_shape.restype = st
    lib.hough_set_timing.argtypes = [P, ctypes.c_int]
    lib.hough_set_timing.restype = st
    lib.hough_timing.argtypes = [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(I64), ctypes.c_int]
    lib.hough_timing.restype = st
    lib.hough_set_event_clock.argtypes = [P, P, I64]
    lib.hough_set_event_clock.restype = st
    lib.hough_clock_rate.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    lib.hough_clock_rate.restype = st
    lib.hough_lds_peak.argtypes = [ctypes.c_int, P, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    lib.hough_lds_peak.restype = st
    lib.hough_graph_create.argtypes = [P, I32, I64, P, P, P, P, I64, P, I64, P, ctypes.POINTER(P)]
    lib.hough_graph_create.restype = st
    lib.hough_graph_launch.argtypes = [P, P]
    lib.hough_graph_launch.restype = st
    lib.hough_graph_destroy.argtypes = [P]
    lib.hough_graph_destroy.restype = st
    lib.hough_autotune.argtypes = [cfgp, ctypes.c_int, P, I32, I64, P, P, P, I32, cfgp,
                                   ctypes.POINTER(ctypes.c_double), ctypes.POINTER(I32)]
    lib.hough_autotune.restype = st
    scfgp = ctypes.POINTER(ServerConfig)
    lib.hough_server_create.argtypes = [cfgp, ctypes.c_int, scfgp, ctypes.POINTER(P)]
    lib.hough_server_create.restype = st
    lib.hough_server_destroy.argtypes = [P]
    lib.hough_server_destroy.restype = st
    lib.hough_server_clock.argtypes = [P]
    lib.hough_server_clock.restype = ctypes.c_double
    lib.hough_server_submit.argtypes = [P, I32, P, P, P, P, P, ctypes.POINTER(I32)]
    lib.hough_server_submit.restype = st
    lib.hough_server_poll.argtypes = [P, I32, P, P, I64, P, I64, ctypes.POINTER(I32)]
    lib.hough_server_poll.restype = st
    lib.hough_server_drain.argtypes = [P, ctypes.c_double]
    lib.hough_server_drain.restype = st
    lib.hough_server_get_stats.argtypes = [P, P]
    lib.hough_server_get_stats.restype = st
    F = ctypes.c_float
    lib.hough_refit_gather.argtypes = [P, I32, P, P, P, P, P, P, P, P, P, P]
    lib.hough_refit_gather.restype = st
    lib.hough_refit_init.argtypes = [P, I32, P, P, P, P, I32, P, P, P, P]
    lib.hough_refit_init.restype = st
    lib.hough_refit_chi2.argtypes = [P, I32, P, P, P, P, I32, P, P, P, F, P]
    lib.hough_refit_chi2.restype = st
    lib.hough_refit_grad.argtypes = [P, I32, P, P, P, P, I32, P, P, P, P, F, P]
    lib.hough_refit_grad.restype = st
    lib.hough_refit_gauss_newton.argtypes = [P, I32, P, P, P, P, I32, P, P, P, P, I32, F, F, P]
    lib.hough_refit_gauss_newton.restype = st
    lib.hough_status_string.argtypes = [ctypes.c_int]
    lib.hough_status_string.restype = ctypes.c_char_p
    lib.hough_last_error.argtypes = [P]
    lib.hough_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _status_string(status: int) -> str:
    try:
        return load_library().hough_status_string(status).decode()
    except Exception:  # library not loadable: plain number
        return str(status)


def default_config(**overrides) -> HoughConfig:
    cfg = HoughConfig()
    load_library().hough_config_default(ctypes.byref(cfg))
    for k, v in overrides.items():
        if not hasattr(cfg, k):
            raise KeyError(k)
        setattr(cfg, k, v)
    return cfg


@dataclasses.dataclass
class FindOutput:
    cand: "object"        # torch uint8 [cap, 40] on the device
    hit_index: "object"   # torch int32 [cap] on the device
    counts: "object"      # torch int64 [8] on the device

    def to_host(self):
        """(candidates as a structured array, hit indices, counts dict)."""
        cnt = self.counts.cpu().numpy()
        info = dict(zip(COUNT_NAMES, (int(x) for x in cnt)))
        nc, nh = info["candidates"], info["hits"]
        cand = self.cand[:nc].cpu().numpy().reshape(-1).view(cand_dtype).copy() if nc else \
            np.zeros(0, cand_dtype)
        hits = self.hit_index[:nh].cpu().numpy().copy()
        return cand, hits, info


class HoughFinder:
    """One library context bound to one device."""

    def __init__(self, device: int = 0, config: Optional[HoughConfig] = None, **overrides):
        import torch  # device memory and streams
        self._torch = torch
        self.lib = load_library()
        self.device = device
        self.config = config if config is not None else default_config(**overrides)
        if config is not None:
            for k, v in overrides.items():
                setattr(self.config, k, v)
        h = ctypes.c_void_p()
        st = self.lib.hough_create(ctypes.byref(self.config), device, ctypes.byref(h))
        if st != HOUGH_OK:
            raise HoughError(st, self.lib.hough_last_error(None).decode())
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self.lib.hough_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _err(self, st: int):
        return HoughError(st, self.lib.hough_last_error(self._h).decode())

    def _stream(self, stream):
        torch = self._torch
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        return ctypes.c_void_p(s.cuda_stream)

    def output_bounds(self, n_events: int, n_hits: int):
        mc = ctypes.c_int64()
        mh = ctypes.c_int64()
        st = self.lib.hough_output_bounds(self._h, n_events, n_hits, ctypes.byref(mc), ctypes.byref(mh))
        if st != HOUGH_OK:
            raise self._err(st)
        return mc.value, mh.value

    def alloc_outputs(self, n_events: int, n_hits: int) -> FindOutput:
        torch = self._torch
        mc, mh = self.output_bounds(n_events, n_hits)
        dev = torch.device("cuda", self.device)
        return FindOutput(torch.empty((max(mc, 1), 40), dtype=torch.uint8, device=dev),
                          torch.empty(max(mh, 1), dtype=torch.int32, device=dev),
                          torch.empty(HOUGH_COUNTS, dtype=torch.int64, device=dev))

    def find(self, z, vane, offsets, out: Optional[FindOutput] = None, stream=None,
             capacities=None, noalloc: bool = False) -> FindOutput:
        """Runs the finder on device tensors z (float32), vane (int16), offsets
        (int64); noalloc selects hough_find_noalloc (the library's fixed
        device scratch instead of the context's workspace; `out` should then
        be given, or this call allocates it)."""
        torch = self._torch
        assert z.dtype == torch.float32 and vane.dtype == torch.int16 and offsets.dtype == torch.int64
        assert z.is_contiguous() and vane.is_contiguous() and offsets.is_contiguous()
        n_events = offsets.numel() - 1
        n_hits = z.numel()
        if out is None:
            out = self.alloc_outputs(n_events, n_hits)
        cc, hc = capacities if capacities is not None else (out.cand.shape[0], out.hit_index.numel())
        fn = self.lib.hough_find_noalloc if noalloc else self.lib.hough_find
        st = fn(self._h, self._stream(stream), n_events, n_hits,
                                 ctypes.c_void_p(offsets.data_ptr()), ctypes.c_void_p(z.data_ptr()),
                                 ctypes.c_void_p(vane.data_ptr()), ctypes.c_void_p(out.cand.data_ptr()), cc,
                                 ctypes.c_void_p(out.hit_index.data_ptr()), hc,
                                 ctypes.c_void_p(out.counts.data_ptr()))
        if st != HOUGH_OK:
            raise self._err(st)
        return out

    def find_host(self, z, vane, offsets):
        """Copies numpy hits to the device, runs, and returns host results."""
        torch = self._torch
        dev = torch.device("cuda", self.device)
        zt = torch.from_numpy(np.ascontiguousarray(z, np.float32)).to(dev)
        vt = torch.from_numpy(np.ascontiguousarray(vane, np.int16)).to(dev)
        ot = torch.from_numpy(np.ascontiguousarray(offsets, np.int64)).to(dev)
        out = self.find(zt, vt, ot)
        torch.cuda.synchronize(dev)
        return out.to_host()

    def debug_accumulator(self, z, vane, iters: int = 0, stream=None):
        """(uint32 numpy [n_theta, n_rho], counts dict) for one event."""
        torch = self._torch
        dev = torch.device("cuda", self.device)
        zt = torch.as_tensor(np.ascontiguousarray(z, np.float32)).to(dev)
        vt = torch.as_tensor(np.ascontiguousarray(vane, np.int16)).to(dev)
        acc = torch.empty(self.config.n_theta * self.config.n_rho, dtype=torch.int32, device=dev)
        counts = torch.empty(HOUGH_COUNTS, dtype=torch.int64, device=dev)
        st = self.lib.hough_debug_accumulator(self._h, self._stream(stream), zt.numel(),
                                              ctypes.c_void_p(zt.data_ptr()), ctypes.c_void_p(vt.data_ptr()),
                                              iters, ctypes.c_void_p(acc.data_ptr()),
                                              ctypes.c_void_p(counts.data_ptr()))
        if st != HOUGH_OK:
            raise self._err(st)
        torch.cuda.synchronize(dev)
        a = acc.cpu().numpy().view(np.uint32).reshape(self.config.n_theta, self.config.n_rho)
        return a, dict(zip(COUNT_NAMES, (int(x) for x in counts.cpu().numpy())))

    def tables(self):
        c = self.config
        cos_t = np.empty(c.n_theta, np.float32)
        sin_t = np.empty(c.n_theta, np.float32)
        phi_v = np.empty(c.n_vanes, np.float32)
        theta_c = np.empty(c.n_theta, np.float32)
        rho_c = np.empty(c.n_rho, np.float32)
        inv_w = np.empty(1, np.float32)
        P = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
        st = self.lib.hough_tables(self._h, P(cos_t), P(sin_t), P(phi_v), P(inv_w), P(theta_c), P(rho_c))
        if st != HOUGH_OK:
            raise self._err(st)
        return cos_t, sin_t, phi_v, inv_w[0], theta_c, rho_c

    def launch_shape(self):
        t = ctypes.c_int32()
        w = ctypes.c_int32()
        l = ctypes.c_int32()  # noqa: E741
        self.lib.hough_launch_shape(self._h, ctypes.byref(t), ctypes.byref(w), ctypes.byref(l))
        return {"tile_rows": t.value, "wg_threads": w.value, "lds_bytes": l.value}

    def tw_find(self, r, z, vane, t, offsets, n_windows: int, tw: Optional[TwConfig] = None, stream=None,
                outputs=None):
        """Time-sliced track finding (hough_tw_find) on device tensors r, z
        (float32), vane (int16), t (float32, sorted per timeline) and CSR
        offsets (int64). Returns (tracks uint8 [cap, 48], hit_index int32,
        counts int64) device tensors; `outputs` reuses such a triple."""
        torch = self._torch
        assert r.dtype == torch.float32 and z.dtype == torch.float32 and t.dtype == torch.float32
        assert vane.dtype == torch.int16 and offsets.dtype == torch.int64
        for x in (r, z, vane, t, offsets):
            assert x.is_contiguous()
        n = z.numel()
        if tw is None:
            tw = tw_config()
        dev = torch.device("cuda", self.device)
        if outputs is None:
            outputs = (torch.empty((max(n // 3, 1), 48), dtype=torch.uint8, device=dev),
                       torch.empty(max(n, 1), dtype=torch.int32, device=dev),
                       torch.empty(HOUGH_COUNTS, dtype=torch.int64, device=dev))
        tr, hi, cnt = outputs
        st = self.lib.hough_tw_find(self._h, self._stream(stream), ctypes.byref(tw), offsets.numel() - 1, n,
                                    ctypes.c_void_p(offsets.data_ptr()), ctypes.c_void_p(r.data_ptr()),
                                    ctypes.c_void_p(z.data_ptr()), ctypes.c_void_p(vane.data_ptr()),
                                    ctypes.c_void_p(t.data_ptr()), int(n_windows), ctypes.c_void_p(tr.data_ptr()),
                                    tr.shape[0], ctypes.c_void_p(hi.data_ptr()), hi.numel(),
                                    ctypes.c_void_p(cnt.data_ptr()))
        if st != HOUGH_OK:
            raise self._err(st)
        return outputs

    def tw_find_host(self, batch, n_windows: Optional[int] = None, tw: Optional[TwConfig] = None):
        """Runs tw_find on a host TimelineBatch; returns (tracks as a
        structured array, hit indices, counts dict)."""
        torch = self._torch
        dev = torch.device("cuda", self.device)
        if n_windows is None:
            n_windows = batch.n_windows(tw.window_ns if tw else 10.0, tw.step_ns if tw else 5.0)
        args = [torch.from_numpy(np.ascontiguousarray(a)).to(dev)
                for a in (batch.r, batch.z, batch.vane, batch.t, batch.offsets)]
        tr, hi, cnt = self.tw_find(*args, n_windows=n_windows, tw=tw)
        torch.cuda.synchronize(dev)
        info = dict(zip(TW_COUNT_NAMES, (int(x) for x in cnt.cpu().numpy())))
        nt, nh = info["tracks"], info["hits"]
        tracks = tr[:nt].cpu().numpy().reshape(-1).view(track_dtype).copy() if nt else np.zeros(0, track_dtype)
        return tracks, hi[:nh].cpu().numpy().copy(), info

    def capture(self, z, vane, offsets, out: Optional[FindOutput] = None) -> "FindGraph":
        """Captures the batched launch for these device tensors (see hough_graph_create)."""
        torch = self._torch
        n_events = offsets.numel() - 1
        n_hits = z.numel()
        if out is None:
            out = self.alloc_outputs(n_events, n_hits)
        g = ctypes.c_void_p()
        st = self.lib.hough_graph_create(self._h, n_events, n_hits, ctypes.c_void_p(offsets.data_ptr()),
                                         ctypes.c_void_p(z.data_ptr()), ctypes.c_void_p(vane.data_ptr()),
                                         ctypes.c_void_p(out.cand.data_ptr()), out.cand.shape[0],
                                         ctypes.c_void_p(out.hit_index.data_ptr()), out.hit_index.numel(),
                                         ctypes.c_void_p(out.counts.data_ptr()), ctypes.byref(g))
        if st != HOUGH_OK:
            raise self._err(st)
        return FindGraph(self, g, out, (z, vane, offsets))

    def set_timing(self, enable: bool):
        self.lib.hough_set_timing(self._h, 1 if enable else 0)

    def set_event_clock(self, stamps=None):
        """Per-event clock stamps into the device uint64/int64 tensor
        `stamps` of 2 * max_events entries ((start, retire) per event) for
        calls of at most max_events events; None turns them off. The tensor
        must stay alive while set."""
        if stamps is None:
            st = self.lib.hough_set_event_clock(self._h, None, 0)
        else:
            assert stamps.is_cuda and stamps.element_size() == 8 and stamps.is_contiguous()
            st = self.lib.hough_set_event_clock(self._h, ctypes.c_void_p(stamps.data_ptr()), stamps.numel() // 2)
        if st != HOUGH_OK:
            raise self._err(st)
        self._clock_buf = stamps

    def timing(self, reset: bool = True):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        st = self.lib.hough_timing(self._h, ctypes.byref(ms), ctypes.byref(n), 1 if reset else 0)
        if st != HOUGH_OK:
            raise self._err(st)
        return ms.value, n.value


class FindGraph:
    """A captured launch; keeps its context and buffers alive."""

    def __init__(self, finder: HoughFinder, handle, out: FindOutput, inputs):
        self.finder = finder
        self._g = handle
        self.out = out
        self._inputs = inputs

    def launch(self, stream=None) -> FindOutput:
        st = self.finder.lib.hough_graph_launch(self._g, self.finder._stream(stream))
        if st != HOUGH_OK:
            raise self.finder._err(st)
        return self.out

    def close(self):
        if getattr(self, "_g", None) is not None and self._g.value:
            self.finder.lib.hough_graph_destroy(self._g)
            self._g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lds_peak(mode: int, device: int = 0, stream=None) -> float:
    """LDS atomic lane operations per second of the device (hough_lds_peak):
    mode 0 conflict-free without return, mode 1 the finder's vote pattern."""
    import torch
    lib = load_library()
    s = stream if stream is not None else torch.cuda.current_stream(device)
    out = ctypes.c_double()
    st = lib.hough_lds_peak(device, ctypes.c_void_p(s.cuda_stream), mode, ctypes.byref(out))
    if st != HOUGH_OK:
        raise HoughError(st, lib.hough_last_error(None).decode())
    return out.value


def clock_rate(device: int = 0) -> float:
    """Ticks per second of the device wall clock the event stamps use."""
    lib = load_library()
    out = ctypes.c_double()
    st = lib.hough_clock_rate(device, ctypes.byref(out))
    if st != HOUGH_OK:
        raise HoughError(st, lib.hough_last_error(None).decode())
    return out.value


def autotune(z, vane, offsets, device: int = 0, repeats: int = 3, stream=None, **overrides):
    """Runs hough_autotune on device tensors; returns (best config, ms per call, shapes tried)."""
    import torch
    lib = load_library()
    base = default_config(**overrides)
    best = HoughConfig()
    ms = ctypes.c_double()
    tried = ctypes.c_int32()
    s = stream if stream is not None else torch.cuda.current_stream(device)
    st = lib.hough_autotune(ctypes.byref(base), device, ctypes.c_void_p(s.cuda_stream), offsets.numel() - 1,
                            z.numel(), ctypes.c_void_p(offsets.data_ptr()), ctypes.c_void_p(z.data_ptr()),
                            ctypes.c_void_p(vane.data_ptr()), repeats, ctypes.byref(best), ctypes.byref(ms),
                            ctypes.byref(tried))
    if st != HOUGH_OK:
        raise HoughError(st, lib.hough_last_error(None).decode())
    return best, ms.value, tried.value


@dataclasses.dataclass
class Served:
    """One finished request: its record (a served_dtype row), candidates and
    hit indices (exactly what a one-event find on the same hits returns)."""
    rec: np.void
    cand: np.ndarray
    hit_index: np.ndarray

    @property
    def tag(self) -> int:
        return int(self.rec["tag"])

    @property
    def status(self) -> int:
        return int(self.rec["status"])

    @property
    def latency(self) -> float:
        return float(self.rec["t_done"] - self.rec["t_arrival"])


class HoughServer:
    """Served form: continuous batching of streamed events over launch lanes
    (hough_server_* in the C ABI). Hits are host numpy arrays; results come
    back as host arrays."""

    def __init__(self, device: int = 0, lanes: int = 0, max_batch_events: int = 0,
                 max_batch_hits: int = 0, queue_hits: int = 0, queue_events: int = 0, device_bytes: int = 0,
                 **cfg_overrides):
        self._lib = load_library()
        self.config = default_config(**cfg_overrides)
        sc = ServerConfig()
        sc.lanes, sc.max_batch_events, sc.max_batch_hits = lanes, max_batch_events, max_batch_hits
        sc.queue_hits, sc.queue_events, sc.device_bytes = queue_hits, queue_events, device_bytes
        h = ctypes.c_void_p()
        st = self._lib.hough_server_create(ctypes.byref(self.config), device, ctypes.byref(sc), ctypes.byref(h))
        if st != HOUGH_OK:
            raise HoughError(st, "hough_server_create")
        self._h = h
        self._cbuf = np.zeros(1 << 16, cand_dtype)
        self._hbuf = np.zeros(1 << 20, np.int32)
        self._rbuf = np.zeros(4096, served_dtype)

    def _grow(self) -> None:
        # the oldest waiting result does not fit the result arrays
        self._cbuf = np.zeros(2 * len(self._cbuf), cand_dtype)
        self._hbuf = np.zeros(2 * len(self._hbuf), np.int32)

    def clock(self) -> float:
        return float(self._lib.hough_server_clock(self._h))

    def submit(self, z: np.ndarray, vane: np.ndarray, offsets: np.ndarray, tags: Optional[np.ndarray] = None,
               t_arrival: Optional[np.ndarray] = None) -> int:
        """Queues the events of a CSR batch (host arrays); returns how many,
        from the first, were taken (fewer only when the queue is full)."""
        z = np.ascontiguousarray(z, np.float32)
        vane = np.ascontiguousarray(vane, np.int16)
        offsets = np.ascontiguousarray(offsets, np.int64)
        n = len(offsets) - 1
        if tags is not None:
            tags = np.ascontiguousarray(tags, np.uint64)
            assert len(tags) == n
        if t_arrival is not None:
            t_arrival = np.ascontiguousarray(t_arrival, np.float64)
            assert len(t_arrival) == n
        acc = ctypes.c_int32()
        ptr = lambda a: a.ctypes.data if a is not None and a.size else None
        st = self._lib.hough_server_submit(self._h, n, ptr(tags), offsets.ctypes.data, ptr(z), ptr(vane),
                                           ptr(t_arrival), ctypes.byref(acc))
        if st != HOUGH_OK:
            raise HoughError(st, "hough_server_submit")
        return int(acc.value)

    def poll(self, max_results: int = 4096) -> list:
        """Finished results, oldest launch first."""
        out = []
        while True:
            if len(self._rbuf) < max_results:
                self._rbuf = np.zeros(max_results, served_dtype)
            k = ctypes.c_int32()
            st = self._lib.hough_server_poll(self._h, max_results, self._rbuf.ctypes.data, self._cbuf.ctypes.data,
                                             len(self._cbuf), self._hbuf.ctypes.data, len(self._hbuf),
                                             ctypes.byref(k))
            if st == HOUGH_ERR_CAPACITY:
                self._grow()
                continue
            if st != HOUGH_OK:
                raise HoughError(st, "hough_server_poll")
            n = k.value
            for r in self._rbuf[:n]:
                c0, nc = int(r["cand_offset"]), int(r["n_candidates"])
                h0, nh = int(r["hit_offset"]), int(r["n_hit_index"])
                out.append(Served(r.copy(), self._cbuf[c0:c0 + nc].copy(), self._hbuf[h0:h0 + nh].copy()))
            if n == 0 or len(out) >= max_results:
                return out
            max_results -= n
            if max_results <= 0:
                return out

    def poll_records(self, max_results: int = 65536):
        """(records, candidates, hit indices) of up to max_results finished
        requests as flat host arrays (offsets in the records)."""
        if len(self._rbuf) < max_results:
            self._rbuf = np.zeros(max_results, served_dtype)
        while True:
            k = ctypes.c_int32()
            st = self._lib.hough_server_poll(self._h, max_results, self._rbuf.ctypes.data, self._cbuf.ctypes.data,
                                             len(self._cbuf), self._hbuf.ctypes.data, len(self._hbuf),
                                             ctypes.byref(k))
            if st == HOUGH_ERR_CAPACITY:
                self._grow()
                continue
            if st != HOUGH_OK:
                raise HoughError(st, "hough_server_poll")
            n = k.value
            recs = self._rbuf[:n].copy()
            nc = int(recs["cand_offset"][-1] + recs["n_candidates"][-1]) if n else 0
            nh = int(recs["hit_offset"][-1] + recs["n_hit_index"][-1]) if n else 0
            return recs, self._cbuf[:nc].copy(), self._hbuf[:nh].copy()

    def drain(self, timeout: float = 60.0) -> None:
        st = self._lib.hough_server_drain(self._h, timeout)
        if st != HOUGH_OK:
            raise HoughError(st, "hough_server_drain (timed out)")

    def stats(self) -> dict:
        a = np.zeros(16, np.int64)
        st = self._lib.hough_server_get_stats(self._h, a.ctypes.data)
        if st != HOUGH_OK:
            raise HoughError(st, "hough_server_get_stats")
        return dict(zip(SERVER_STAT_NAMES, (int(x) for x in a)))

    def close(self) -> None:
        if getattr(self, "_h", None):
            self._lib.hough_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Helix refit (hough_refit_* in the C ABI)
# ---------------------------------------------------------------------------

REFIT_SIGMA_MM = 0.055
REFIT_STEPS = 20
REFIT_DAMPING = 1e-3


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _check(st, what):
    if st != HOUGH_OK:
        raise HoughError(st, what)


@dataclasses.dataclass
class RefitHits:
    """Device arrays of the candidates' hits (CSR) and the per-hit state the
    initial fit sets (root sign and reference turning angle)."""
    offsets: "object"     # int64 [n_cand + 1]
    r: "object"           # float32 [n_hits]
    z: "object"
    vane: "object"        # int16
    n_vanes: int = 40
    sign: "object" = None
    aref: "object" = None
    status: "object" = None

    @property
    def n_cand(self) -> int:
        return int(self.offsets.numel()) - 1


def refit_gather(out: "FindOutput", offsets, r, z, vane, stream=None, n_vanes: int = 40) -> RefitHits:
    """The hits of the candidates in a find call's output (device tensors of
    the same batch) as a RefitHits."""
    import torch
    lib = load_library()
    cnt = out.counts.cpu().numpy()
    n_cand, n_hit = int(cnt[0]), int(cnt[1])
    dev = z.device
    off = torch.empty(n_cand + 1, dtype=torch.int64, device=dev)
    ro = torch.empty(max(n_hit, 1), dtype=torch.float32, device=dev)
    zo = torch.empty_like(ro)
    vo = torch.empty(max(n_hit, 1), dtype=torch.int16, device=dev)
    s = _stream_ptr(stream, dev)
    _check(lib.hough_refit_gather(s, n_cand, _ptr(out.cand), _ptr(out.hit_index), _ptr(offsets), _ptr(r), _ptr(z),
                                  _ptr(vane), _ptr(off), _ptr(ro), _ptr(zo), _ptr(vo)), "hough_refit_gather")
    return RefitHits(off, ro[:n_hit], zo[:n_hit], vo[:n_hit], n_vanes)


def _stream_ptr(stream, dev):
    import torch
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    return ctypes.c_void_p(st.cuda_stream)


def refit_init(h: RefitHits, stream=None):
    """Initial parameters (float32 [n_cand, 5]); sets h.sign, h.aref, h.status."""
    import torch
    lib = load_library()
    dev = h.r.device
    n = h.n_cand
    params = torch.zeros((max(n, 1), 5), dtype=torch.float32, device=dev)
    h.sign = torch.empty(max(h.r.numel(), 1), dtype=torch.float32, device=dev)
    h.aref = torch.empty_like(h.sign)
    h.status = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    _check(lib.hough_refit_init(_stream_ptr(stream, dev), n, _ptr(h.offsets), _ptr(h.r), _ptr(h.z), _ptr(h.vane),
                                h.n_vanes, _ptr(params), _ptr(h.sign), _ptr(h.aref), _ptr(h.status)),
           "hough_refit_init")
    return params[:n]


def refit_chi2(h: RefitHits, params, sigma: float = REFIT_SIGMA_MM, stream=None):
    import torch
    lib = load_library()
    params = params.contiguous()
    chi2 = torch.empty(max(h.n_cand, 1), dtype=torch.float32, device=params.device)
    _check(lib.hough_refit_chi2(_stream_ptr(stream, params.device), h.n_cand, _ptr(h.offsets), _ptr(h.r), _ptr(h.z),
                                _ptr(h.vane), h.n_vanes, _ptr(h.sign), _ptr(h.aref), _ptr(params), sigma,
                                _ptr(chi2)), "hough_refit_chi2")
    return chi2[:h.n_cand]


def refit_grad(h: RefitHits, params, grad_chi2=None, sigma: float = REFIT_SIGMA_MM, stream=None):
    import torch
    lib = load_library()
    params = params.contiguous()
    g = torch.empty_like(params)
    if grad_chi2 is not None:
        grad_chi2 = grad_chi2.contiguous().to(torch.float32)
    _check(lib.hough_refit_grad(_stream_ptr(stream, params.device), h.n_cand, _ptr(h.offsets), _ptr(h.r), _ptr(h.z),
                                _ptr(h.vane), h.n_vanes, _ptr(h.sign), _ptr(h.aref), _ptr(params),
                                _ptr(grad_chi2), sigma, _ptr(g)), "hough_refit_grad")
    return g


def refit_gauss_newton(h: RefitHits, params, steps: int = REFIT_STEPS, damping: float = REFIT_DAMPING,
                       sigma: float = REFIT_SIGMA_MM, stream=None):
    """Gauss-Newton steps on params in place; returns the final chi^2."""
    import torch
    lib = load_library()
    assert params.is_contiguous() and params.dtype == torch.float32
    chi2 = torch.empty(max(h.n_cand, 1), dtype=torch.float32, device=params.device)
    _check(lib.hough_refit_gauss_newton(_stream_ptr(stream, params.device), h.n_cand, _ptr(h.offsets), _ptr(h.r),
                                        _ptr(h.z), _ptr(h.vane), h.n_vanes, _ptr(h.sign), _ptr(h.aref),
                                        _ptr(h.status), _ptr(params), steps, damping, sigma, _ptr(chi2)),
           "hough_refit_gauss_newton")
    return chi2[:h.n_cand]


def _autograd_function():
    import torch

    class HelixChi2(torch.autograd.Function):
        """chi^2 per candidate as a differentiable function of the helix
        parameters: forward by the chi^2 kernel, backward by the hand-written
        adjoint kernel."""

        @staticmethod
        def forward(ctx, params, hits: RefitHits, sigma: float = REFIT_SIGMA_MM):
            params = params.detach().contiguous()
            ctx.hits = hits
            ctx.sigma = sigma
            ctx.save_for_backward(params)
            return refit_chi2(hits, params, sigma)

        @staticmethod
        def backward(ctx, grad_out):
            (params,) = ctx.saved_tensors
            return refit_grad(ctx.hits, params, grad_out, ctx.sigma), None, None

    return HelixChi2


_HELIX_CHI2 = None


def helix_chi2(params, hits: RefitHits, sigma: float = REFIT_SIGMA_MM):
    """Differentiable chi^2 per candidate (torch.autograd.Function)."""
    global _HELIX_CHI2
    if _HELIX_CHI2 is None:
        _HELIX_CHI2 = _autograd_function()
    return _HELIX_CHI2.apply(params, hits, sigma)


def momentum_mev(params, b_tesla: float = 3.0):
    """|p| in MeV/c from fitted parameters (tensor [n, 5])."""
    pt = 0.299792458 * b_tesla / params[:, 0].abs()
    return pt * (1.0 + params[:, 4] * params[:, 4]).sqrt()
