"""Benchmark: Hough track finding at pileup 50 on one MI355X.

One step = one call of the finder (the whole find-and-remove hot path) over a
batch of 4096 synthetic pileup-50 events already resident in HBM (1024 x 1024
uint32 histogram, T = 6, window peaks with w = 1). Reports batched events/s
as the value, and beside it:
  * the plain one-event-per-call rate and latency percentiles;
  * the finder kernel's roofline figures: VALU ("roofline"), the LDS atomic
    rate of its votes against the device's measured rate ("lds_roofline"),
    HBM traffic from the committed rocprofv3 counter summary;
  * the CPU oracle on one core and on every core of the host's share, both
    before the GPU is touched;
  * the Eq. (5) track-finding efficiency on the generator truth;
  * the served stream, the helix refit and the coarse-to-fine search legs.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--plain-events P]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "events/s Hough track-finding at pileup 50 (batched vs plain) + p99 event latency"
N_EVENTS = 4096
PILEUP = 50
# unfused, unpacked float32 operations of Eq. (4) and its binning per vote:
# phi*c, z*s, add, subtract rho_min, multiply by inv_w
FLOPS_PER_VOTE = 5
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one float op per lane per clock
VALU_PEAK_TFLOPS = 256 * 64 * 2.4e9 / 1e12


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def host_cpu_info():
    """CPU model and the cores this process may use (the oracle's host)."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cores": usable}


def event_mismatches(got_cand, got_hits, want):
    """Events whose candidates (every field) or ordered hit lists differ
    between a finder output and the oracle's; 0 means the two outputs are
    byte-identical."""
    import numpy as np
    if (len(got_cand) == len(want.cand) and len(got_hits) == len(want.hit_index)
            and np.array_equal(got_cand.view(np.uint8), want.cand.view(np.uint8))
            and np.array_equal(got_hits, want.hit_index)):
        return 0
    evs = np.union1d(np.unique(got_cand["event"]), np.unique(want.cand["event"]))
    bad = 0
    for e in evs:
        a = got_cand[got_cand["event"] == e]
        b = want.cand[want.cand["event"] == e]
        if len(a) != len(b) or any(not np.array_equal(a[f], b[f]) for f in a.dtype.names if f != "hit_offset"):
            bad += 1
            continue
        if len(a):
            ha = got_hits[a["hit_offset"][0]:a["hit_offset"][0] + int(a["n_hits"].sum())]
            hb = want.hit_index[b["hit_offset"][0]:b["hit_offset"][0] + int(b["n_hits"].sum())]
            bad += int(not np.array_equal(ha, hb))
    return bad


def parity_record(got_cand, got_hits, want, n_events):
    return {"events": n_events, "candidates": len(got_cand), "hits": len(got_hits),
            "oracle_candidates": len(want.cand), "oracle_hits": len(want.hit_index),
            "mismatched_events": event_mismatches(got_cand, got_hits, want), "check": "byte-equal, every event"}


def timed_batched(f, z, vane, offs, out, stream, steps, warmup):
    """(ms per call from the host clock, finder kernel ms per launch from HIP
    events on the launch stream) over `steps` calls after `warmup` calls."""
    import torch
    for _ in range(warmup):
        f.find(z, vane, offs, out=out, stream=stream)
    torch.cuda.synchronize()
    f.set_timing(True)
    f.timing(reset=True)
    t1 = time.perf_counter()
    for _ in range(steps):
        f.find(z, vane, offs, out=out, stream=stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t1
    f.set_timing(False)
    kern_ms, launches = f.timing(reset=True)
    return 1e3 * wall / steps, kern_ms / max(launches, 1)


def event_latency(f, z, vane, offs, out, stream, n_events, repeats):
    """Per-event latency of the batched call from device clock stamps: an
    event's retire stamp (its finder workgroup wrote its last output) minus
    the call's first finder workgroup start, over `repeats` calls."""
    import numpy as np
    import torch
    from paper_2511_02742_amd.hough import clock_rate
    rate = clock_rate(0)
    stamps = torch.zeros(2 * n_events, dtype=torch.int64, device=z.device)
    f.set_event_clock(stamps)
    lat, spans = [], []
    try:
        for _ in range(repeats):
            stamps.zero_()
            f.find(z, vane, offs, out=out, stream=stream)
            torch.cuda.synchronize()
            s = stamps.cpu().numpy().reshape(-1, 2).astype(np.float64)
            t0 = s[:, 0].min()
            lat.append((s[:, 1] - t0) / rate)
            spans.append((s[:, 1].max() - t0) / rate)
    finally:
        f.set_event_clock(None)
    lat = np.concatenate(lat)
    return {"latency_us_p50": round(1e6 * float(np.percentile(lat, 50)), 2),
            "latency_us_p99": round(1e6 * float(np.percentile(lat, 99)), 2),
            "latency_us_max": round(1e6 * float(lat.max()), 2),
            "device_span_us_median": round(1e6 * float(np.median(spans)), 2),
            "calls": repeats, "clock_hz": rate,
            "definition": "retire stamp of each event (its finder workgroup wrote its last output) minus the "
                          "call's first finder-workgroup start; device wall clock"}


def graph_legs(f, batch, z, vane, offs, stream, steps, warmup, want):
    """The batched call captured in a HIP graph: replays on device-resident
    hits, and the whole transfer-inclusive round (pinned host hits to the
    device, replay, counts and the exact outputs back to pinned host memory)
    as the paper's timings count host-device copies (Table 1)."""
    import numpy as np
    import torch
    g = f.capture(z, vane, offs)
    for _ in range(warmup):
        g.launch(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(steps):
        g.launch(stream)
    torch.cuda.synchronize()
    replay_ms = 1e3 * (time.perf_counter() - t1) / steps
    cand, hits, info = g.out.to_host()
    par = parity_record(cand, hits, want, len(batch.offsets) - 1) if want is not None else None
    hz = torch.from_numpy(batch.z).pin_memory()
    hv = torch.from_numpy(batch.vane).pin_memory()
    ho = torch.from_numpy(batch.offsets).pin_memory()
    hcnt = torch.empty(g.out.counts.shape, dtype=torch.int64).pin_memory()
    hcand = torch.empty(g.out.cand.shape, dtype=torch.uint8).pin_memory()
    hhits = torch.empty(g.out.hit_index.shape, dtype=torch.int32).pin_memory()

    def round_trip():
        z.copy_(hz, non_blocking=True)
        vane.copy_(hv, non_blocking=True)
        offs.copy_(ho, non_blocking=True)
        g.launch(stream)
        hcnt.copy_(g.out.counts, non_blocking=True)
        stream.synchronize()
        nc, nh = int(hcnt[0]), int(hcnt[1])
        hcand[:nc].copy_(g.out.cand[:nc], non_blocking=True)
        hhits[:nh].copy_(g.out.hit_index[:nh], non_blocking=True)
        stream.synchronize()
    for _ in range(warmup):
        round_trip()
    t1 = time.perf_counter()
    for _ in range(steps):
        round_trip()
    rt_ms = 1e3 * (time.perf_counter() - t1) / steps
    nc, nh = int(hcnt[0]), int(hcnt[1])
    rt_ok = (want is not None and nc == len(want.cand) and nh == len(want.hit_index)
             and np.array_equal(hcand[:nc].numpy().reshape(-1), want.cand.view(np.uint8).reshape(-1))
             and np.array_equal(hhits[:nh].numpy(), want.hit_index))
    g.close()
    ne = len(batch.offsets) - 1
    return {"replay": {"events_per_s": round(ne / (replay_ms * 1e-3), 1), "ms_per_call": round(replay_ms, 4),
                       "parity": par},
            "with_transfers": {"events_per_s": round(ne / (rt_ms * 1e-3), 1), "ms_per_call": round(rt_ms, 4),
                               "h2d_bytes": int(batch.z.nbytes + batch.vane.nbytes + batch.offsets.nbytes),
                               "d2h_bytes": int(16 * 8 + 40 * nc + 4 * nh),
                               "outputs_byte_equal_oracle": bool(rt_ok),
                               "note": "pinned host hits -> device, graph replay, counts back, then exactly the "
                                       "candidates and hit lists back; two stream synchronisations per call"}}


def oracle_references(jobs, log):
    """The oracle's full outputs for every event of each (name, config,
    batch) job, in independent processes over event slices (the unchanged
    single-threaded oracle in each)."""
    from oracle.oracle import oracle_find_batch_sliced
    workers = max(1, min(16, os.cpu_count() or 1))
    refs = {}
    for name, ocfg, b in jobs:
        t0 = time.perf_counter()
        refs[name] = oracle_find_batch_sliced(ocfg, b.offsets, b.z, b.vane, workers=workers)
        log("oracle reference %s: %d candidates, %d hits in %.1f s"
            % (name, len(refs[name].cand), len(refs[name].hit_index), time.perf_counter() - t0))
    return refs


def cpu_sample(ocfg, batch, seconds, label):
    """The single-threaded oracle over the first events of `batch` for about
    `seconds` (at least 16 events): events/s and per-event p50/p99."""
    import numpy as np
    from oracle import oracle_find
    n_ev = len(batch.offsets) - 1
    n_done = 0
    per = []
    tc0 = time.perf_counter()
    while n_done < n_ev and (time.perf_counter() - tc0 < seconds or n_done < 16):
        lo, hi = int(batch.offsets[n_done]), int(batch.offsets[n_done + 1])
        ts = time.perf_counter()
        oracle_find(ocfg, batch.z[lo:hi], batch.vane[lo:hi], event_id=n_done)
        per.append(time.perf_counter() - ts)
        n_done += 1
    tc = time.perf_counter() - tc0
    per = np.array(per)
    return {"value": round(n_done / tc, 2), "unit": "events/s", "cores": 1, "kind": "oracle",
            "sample": "first %d of the same %d %s events, one thread, %.1f s" % (n_done, n_ev, label, tc),
            "latency_us_p50": round(1e6 * float(np.percentile(per, 50)), 1),
            "latency_us_p99": round(1e6 * float(np.percentile(per, 99)), 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--plain-events", type=int, default=512)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle timings and the oracle references (no parity check then)")
    ap.add_argument("--no-autotune", action="store_true", help="headline on the library's default shape")
    ap.add_argument("--launch", default="",
                    help="WG,TILE: headline on this finder workgroup size and tile rows instead of the autotuner's "
                         "pick (for profiler runs of one shape)")
    ap.add_argument("--serve-events", type=int, default=1000000,
                    help="requests per offered rate in the served-stream leg (0: skip it)")
    ap.add_argument("--serve-rates", default="20000,50000,100000")
    ap.add_argument("--serve-lanes", type=int, default=3)
    ap.add_argument("--serve-pool", type=int, default=4096)
    ap.add_argument("--refit-events", type=int, default=4096,
                    help="events of the Poisson(20) batch whose candidates the refit leg fits (0: skip it)")
    ap.add_argument("--refit-oracle", type=int, default=30,
                    help="pure candidates also fitted by the float64 oracle for the parameter error")
    ap.add_argument("--no-coarse-fine", action="store_true",
                    help="skip the coarse-to-fine leg (the paper's 18 x 100 -> 10 x 10 histograms)")
    ap.add_argument("--tw-timelines", type=int, default=64,
                    help="timelines of 10^4 decays per rate in the time-sliced leg (0: skip it)")
    ap.add_argument("--tw-rates", default="6.0,0.6,0.06", help="decay rates (per ns) of the time-sliced leg")
    ap.add_argument("--only-batched", action="store_true",
                    help="the batched headline leg alone (for profiler runs): no oracle, plain, graph, cfg3, "
                         "served, refit or coarse-to-fine legs")
    ap.add_argument("--finder", choices=("nms", "cf"), default="nms",
                    help="with --only-batched: the full-grid finder on 1024x1024 (nms) or the coarse-to-fine "
                         "finder on 180x1000 (cf) on the same events")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one device-to-device copy of this size first, as the reference kernel for "
                         "FETCH_SIZE / WRITE_SIZE counter scaling")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(events shard across GPUs with no communication between them).", file=sys.stderr)
        sys.exit(2)
    if args.only_batched:
        args.no_cpu_baseline = True
        args.tw_timelines = 0
        args.serve_events = 0
        args.refit_events = 0
        args.no_coarse_fine = True

    import numpy as np

    from oracle import OracleConfig
    from paper_2511_02742_amd import eventgen

    t0 = time.time()
    batch = eventgen.pileup_batch(N_EVENTS, n_tracks=PILEUP, seed0=0)
    log("generated %d events in %.1f s: %s" % (N_EVENTS, time.time() - t0, eventgen.hit_histogram(batch)))
    b3 = None if args.only_batched else eventgen.poisson_batch(N_EVENTS)

    # ---- CPU oracle: timings on bounded samples and the full references
    # for the parity checks, all before anything touches the GPU (the
    # all-cores figures start worker processes)
    cpu = cpu_all = cpu3 = None
    refs = {}
    host = host_cpu_info()
    if not args.no_cpu_baseline:
        cpu = cpu_sample(OracleConfig(), batch, args.cpu_seconds, "pileup-50")
        cpu.update(host)
        log("cpu oracle: %s" % cpu)
        cpu_all = oracle_all_cores(batch, args.cpu_seconds, log)
        cpu_all.update(host)
        cpu3 = cpu_sample(OracleConfig(), b3, args.cpu_seconds / 3, "Poisson(20)")
        log("cpu oracle, Poisson(20) batch: %s" % cpu3)
        jobs = [("pileup50", OracleConfig(), batch), ("poisson20", OracleConfig(), b3)]
        if not args.no_coarse_fine:
            for name, mode in (("coarse_fine", 2), ("argmax", 0), ("nms", 1)):
                jobs.append(("cf_" + name, OracleConfig(n_theta=180, n_rho=1000, peak_mode=mode), batch))
        refs = oracle_references(jobs, log)
    tw_in = tw_inputs(args, log) if args.tw_timelines > 0 else None

    import torch

    from paper_2511_02742_amd.hough import COUNT_NAMES, HoughFinder, autotune

    dev = torch.device("cuda", 0)
    z = torch.from_numpy(batch.z).to(dev)
    vane = torch.from_numpy(batch.vane).to(dev)
    offs = torch.from_numpy(batch.offsets).to(dev)

    if args.copy_calibration_mib > 0:
        nb = args.copy_calibration_mib << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        # An elementwise kernel (not a DMA memcpy, which the counters miss)
        # that reads and writes exactly nb bytes each.
        torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize(dev)
        log("copy calibration (MulFunctor kernel): %d bytes read, %d bytes written" % (nb, nb))
        del src, dst

    stream = torch.cuda.current_stream(dev)
    # ---- launch shape: the autotuner on this batch (its time is reported
    # apart and never counted in events/s)
    tune = None
    if args.only_batched and args.finder == "cf":
        f = HoughFinder(0, n_theta=180, n_rho=1000, peak_mode=2)
    elif args.launch:
        wg, tr = (int(x) for x in args.launch.split(","))
        f = HoughFinder(0, wg_threads=wg, tile_rows=tr)
    elif args.no_autotune:
        f = HoughFinder(0)
    else:
        tt0 = time.perf_counter()
        best, best_ms, tried = autotune(z, vane, offs, repeats=3)
        tune = {"seconds": round(time.perf_counter() - tt0, 3), "shapes_tried": tried,
                "best_ms_per_call": round(best_ms, 4),
                "best": {k: int(getattr(best, k)) for k in ("wg_threads", "sweep_groups", "sweep_threads",
                                                             "tile_rows")}}
        log("autotune: %s" % tune)
        f = HoughFinder(0, config=best)
    shape = f.launch_shape()
    out = f.alloc_outputs(N_EVENTS, batch.n_hits)

    # ---- batched: one call over all events --------------------------------
    ms_per_step, kern_avg_ms = timed_batched(f, z, vane, offs, out, stream, args.steps, args.warmup)
    info = dict(zip(COUNT_NAMES, (int(x) for x in out.counts.cpu().numpy())))
    assert info["status"] == 0, info
    main_cand, main_hits, _ = out.to_host()
    value = 1e3 * N_EVENTS / ms_per_step
    log("batched: %.3f ms/step, %.0f events/s, finder kernel %.3f ms avg" % (ms_per_step, value, kern_avg_ms))
    parity = parity_record(main_cand, main_hits, refs["pileup50"], N_EVENTS) if "pileup50" in refs else None
    log("parity: %s" % parity)
    lat_b = event_latency(f, z, vane, offs, out, stream, N_EVENTS, 10)
    log("batched per-event latency: %s" % lat_b)

    if args.only_batched:
        print(json.dumps({"metric": METRIC, "value": round(value, 1), "unit": "events/s", "n_gpus": 1,
                          "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
                          "kernel_avg_ms": round(kern_avg_ms, 4), "launch": shape, "autotune": tune,
                          "finder": args.finder, "only_batched": True}), flush=True)
        return

    eff = eq5_efficiency(batch, main_cand, main_hits)
    log("Eq. (5) efficiency: %s" % eff)
    graph = graph_legs(f, batch, z, vane, offs, stream, args.steps, args.warmup, refs.get("pileup50"))
    log("graph: %s" % graph)

    # ---- plain: one event per call, the library's default shape ----------
    fp = HoughFinder(0)
    npl = min(args.plain_events, N_EVENTS)
    single = []
    for e in range(npl):
        lo, hi = int(batch.offsets[e]), int(batch.offsets[e + 1])
        o = torch.tensor([0, hi - lo], dtype=torch.int64, device=dev)
        single.append((z[lo:hi], vane[lo:hi], o, fp.alloc_outputs(1, hi - lo)))
    for e in range(min(16, npl)):
        zz, vv, oo, oo_out = single[e]
        fp.find(zz, vv, oo, out=oo_out, stream=stream)
    torch.cuda.synchronize(dev)
    lat = np.zeros(npl)
    tp0 = time.perf_counter()
    for e in range(npl):
        zz, vv, oo, oo_out = single[e]
        ts = time.perf_counter()
        fp.find(zz, vv, oo, out=oo_out, stream=stream)
        stream.synchronize()
        lat[e] = time.perf_counter() - ts
    tp1 = time.perf_counter()
    plain_rate = npl / (tp1 - tp0)
    plain_bad = 0
    if "pileup50" in refs:
        want = refs["pileup50"]
        for e in range(npl):
            c, h, _ = single[e][3].to_host()
            sel = want.cand["event"] == e
            wc = want.cand[sel].copy()
            wh = want.hit_index[wc["hit_offset"][0]:wc["hit_offset"][0] + int(wc["n_hits"].sum())] if len(wc) \
                else want.hit_index[:0]
            wc["event"] = 0
            if len(wc):
                wc["hit_offset"] -= wc["hit_offset"][0]
            plain_bad += int(not (np.array_equal(c.view(np.uint8), wc.view(np.uint8)) and np.array_equal(h, wh)))
    log("plain: %.0f events/s, p50 %.1f us, p99 %.1f us, %d mismatched events"
        % (plain_rate, 1e6 * np.percentile(lat, 50), 1e6 * np.percentile(lat, 99), plain_bad))

    # ---- the uneven Poisson(20) batch -------------------------------------
    z3 = torch.from_numpy(b3.z).to(dev)
    v3 = torch.from_numpy(b3.vane).to(dev)
    o3 = torch.from_numpy(b3.offsets).to(dev)
    out3 = f.alloc_outputs(N_EVENTS, b3.n_hits)
    ms3, k3 = timed_batched(f, z3, v3, o3, out3, stream, args.steps, args.warmup)
    c3, h3, i3 = out3.to_host()
    lens3 = np.diff(b3.offsets)
    poisson = {"workload": "%d events, tracks ~ Poisson(20) clipped to [1, 100] + 1%% noise, seeds 1000000.., "
                           "1024x1024, T=6, nms w=1" % N_EVENTS,
               "hits_total": int(b3.n_hits), "hits_per_event_mean": round(float(lens3.mean()), 1),
               "hits_per_event_range": [int(lens3.min()), int(lens3.max())],
               "events_per_s": round(1e3 * N_EVENTS / ms3, 1), "ms_per_step": round(ms3, 4),
               "kernel_avg_ms": round(k3, 4), "candidates": i3["candidates"],
               "parity": parity_record(c3, h3, refs["poisson20"], N_EVENTS) if "poisson20" in refs else None,
               "cpu_baseline": cpu3,
               "event_latency": event_latency(f, z3, v3, o3, out3, stream, N_EVENTS, 5)}
    log("Poisson(20) batch: %s" % poisson)

    # ---- HBM traffic of the finder kernel from the committed counter summary
    # (reported only while the kernel source still matches the one profiled)
    traffic = profiled_traffic("k_find_pileup50", "hough_kernels.hip")

    # ---- LDS atomic roofline of the finder's votes: every histogram vote is
    # one LDS atomic add. The method's votes (N_theta x the alive hits of
    # every iteration's histogram, the oracle's count) are the work; the
    # kernel's own atomics (fewer: later histograms are recounted from the
    # hot set) are reported beside them.
    from paper_2511_02742_amd.hough import lds_peak
    peak_cf = lds_peak(0)
    peak_vote = lds_peak(1)
    method_votes = refs["pileup50"].votes if "pileup50" in refs else None
    work = method_votes if method_votes is not None else info["votes"]
    votes_s = work / (kern_avg_ms * 1e-3)
    lds = {"bound": "lds", "achieved": round(votes_s, 1), "unit": "votes/s (lane LDS atomics)",
           "peak": round(peak_cf, 1), "frac": round(votes_s / peak_cf, 4),
           "peak_vote_pattern": round(peak_vote, 1), "frac_vote_pattern": round(votes_s / peak_vote, 4),
           "method_votes_per_launch": method_votes, "kernel_votes_per_launch": info["votes"],
           "kernel_votes_frac": round(info["votes"] / (kern_avg_ms * 1e-3) / peak_cf, 4),
           "kernel": "k_find", "kernel_avg_ms": round(kern_avg_ms, 4),
           "note": "work: the method's votes, N_theta x alive hits summed over every iteration's histogram "
                   "(oracle count); peak: conflict-free ds_add_u32 without return; vote pattern: random bins "
                   "of a 1024-word row with return (hough_lds_peak, measured in this run)"}
    log("LDS roofline: %s" % lds)
    # the same work against the unfused float VALU issue rate: 5 rounded
    # float operations of Eq. (4) per vote
    achieved = FLOPS_PER_VOTE * work / (kern_avg_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 4), "peak": round(VALU_PEAK_TFLOPS, 2),
                "unit": "TFLOP/s", "frac": round(achieved / VALU_PEAK_TFLOPS, 4), "traffic": traffic,
                "kernel": "k_find", "kernel_avg_ms": round(kern_avg_ms, 4),
                "method_votes_per_launch": method_votes, "flops_per_vote": FLOPS_PER_VOTE,
                "kernel_evals_per_launch": info["evals"],
                "lds_frac": lds["frac"], "lds_frac_vote_pattern": lds["frac_vote_pattern"]}

    tw = tw_bench(args, tw_in, log) if tw_in else None
    served = serve_bench(args, f, log) if args.serve_events > 0 else None
    refit = refit_bench(args, f, log) if args.refit_events > 0 else None
    coarse_fine = None if args.no_coarse_fine else coarse_fine_bench(args, batch, z, vane, offs, log, peak_vote,
                                                                     refs)

    rec = {
        "metric": METRIC, "value": round(value, 1), "unit": "events/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "pileup-50 batch: %d events x 50 helix tracks + 1%% noise, seeds 0..%d, "
                               "1024x1024 uint32 histogram, T=6, nms w=1" % (N_EVENTS, N_EVENTS - 1),
                   "n_events": N_EVENTS, "hits_total": batch.n_hits, "n_theta": 1024, "n_rho": 1024,
                   "min_votes": 6, "peak_mode": "nms", "launch": shape},
        "parity": parity,
        "autotune": tune,
        "batched_ms_per_launch": round(ms_per_step, 4),
        "batched_event_latency": lat_b,
        "graph": graph,
        "plain": {"value": round(plain_rate, 1), "unit": "events/s", "events": npl,
                  "latency_us_p50": round(1e6 * float(np.percentile(lat, 50)), 2),
                  "latency_us_p99": round(1e6 * float(np.percentile(lat, 99)), 2),
                  "mismatched_events": plain_bad if refs else None},
        "speedup_batched_vs_plain": round(value / plain_rate, 2),
        "work": {k: info[k] for k in ("candidates", "hits", "evals", "votes", "iters", "max_iters", "passes",
                                      "tiled", "truncations", "hot_scans", "hotset_full", "recounts", "ordered")},
        "efficiency_eq5": eff,
        "roofline": roofline,
        "lds_roofline": lds,
        "cpu_baseline": cpu,
        "cpu_baseline_all_cores": cpu_all,
        "poisson20": poisson,
        "time_windows": tw,
        "served": served,
        "refit": refit,
        "coarse_fine": coarse_fine,
    }
    print(json.dumps(rec), flush=True)


TW_DECAYS = 10000        # decays per timeline (the size of the paper's Table 1 runs)
TW_CHECKED = 2           # timelines per rate also run by the oracle


def _tw_oracle_job(job):
    from oracle import OracleConfig, TwConfig, oracle_tw_find_batch
    rate, offsets, r, z, vane, t, n_windows = job
    t0 = time.perf_counter()
    res = oracle_tw_find_batch(OracleConfig(), TwConfig(), offsets, r, z, vane, t, n_windows)
    return rate, res, time.perf_counter() - t0


def tw_inputs(args, log):
    """Timelines of the time-sliced leg, and the oracle on the first ones of
    each rate (independent processes, one per job; before the GPU is used)."""
    import multiprocessing as mp
    from paper_2511_02742_amd import eventgen
    rates = [float(x) for x in args.tw_rates.split(",") if x]
    t0 = time.perf_counter()
    batches = {rate: eventgen.timeline_batch(args.tw_timelines, rate, TW_DECAYS / rate,
                                            seed0=4_000_000 + 1000 * int(round(rate * 100)))
               for rate in rates}
    log("time-sliced leg: generated %d timelines x %d rates in %.1f s" % (args.tw_timelines, len(rates),
                                                                        time.perf_counter() - t0))
    refs = {}
    if not args.no_cpu_baseline:
        jobs = []
        for rate, b in batches.items():
            k = min(TW_CHECKED, b.n_timelines)
            hi = int(b.offsets[k])
            jobs.append((rate, b.offsets[:k + 1].copy(), b.r[:hi].copy(), b.z[:hi].copy(), b.vane[:hi].copy(),
                         b.t[:hi].copy(), b.n_windows()))
        with mp.get_context("spawn").Pool(len(jobs)) as pool:
            for rate, res, sec in pool.map(_tw_oracle_job, jobs):
                refs[rate] = (res, sec)
                log("time-sliced oracle, %g decays/ns: %d tracks in %.1f s" % (rate, len(res.tracks), sec))
    return batches, refs


def tw_bench(args, tw_in, log):
    """Time-sliced track finding (10 ns windows sliding by 5 ns, Hough seeds
    per window, three-hit seeds extended across vanes, flagged tracks
    continued) on timelines of 10^4 decays at the paper's decay rates:
    decays/s and windows/s of one call over all timelines, the first
    timelines byte-checked against the oracle, and the oracle's own rate on
    one core."""
    import numpy as np
    import torch
    from paper_2511_02742_amd.hough import TW_COUNT_NAMES, HoughFinder, track_dtype, tw_config
    batches, refs = tw_in
    dev = torch.device("cuda", 0)
    f = HoughFinder(0)
    tw = tw_config()
    out = {"workload": "%d timelines per rate, %d muon decays each (Poisson times over 10^4 / rate ns), "
                       "50-track-equivalent geometry, 1%% noise; 10 ns windows, 5 ns step; 1024x1024 Hough "
                       "seeds, T=6, nms w=1" % (args.tw_timelines, TW_DECAYS), "rates": []}
    for rate, b in batches.items():
        nw = b.n_windows()
        ts = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (b.r, b.z, b.vane, b.t, b.offsets)]
        outs = None
        reps = 1 if nw > 10000 else 3
        times = []
        for i in range(reps + 1):
            torch.cuda.synchronize(dev)
            t0 = time.perf_counter()
            outs = f.tw_find(*ts, n_windows=nw, tw=tw, outputs=outs)
            torch.cuda.synchronize(dev)
            if i > 0:
                times.append(time.perf_counter() - t0)
        sec = float(np.median(times))
        info = dict(zip(TW_COUNT_NAMES, (int(x) for x in outs[2].cpu().numpy())))
        assert info["status"] == 0, info
        n_dec = sum(len(tl.t_decay) for tl in b.timelines)
        ent = {"decays_per_ns": rate, "timelines": b.n_timelines, "decays": n_dec, "hits": b.n_hits,
               "windows_per_timeline": nw, "seconds_per_call": round(sec, 4),
               "decays_per_s": round(n_dec / sec, 1), "windows_per_s": round(b.n_timelines * nw / sec, 1),
               "tracks": info["tracks"], "track_hits": info["hits"], "hough_candidates": info["candidates"],
               "continuations": info["continued"]}
        if rate in refs:
            res, osec = refs[rate]
            nt, nh = len(res.tracks), len(res.hit_index)
            g_tr = outs[0][:nt].cpu().numpy().reshape(-1).view(track_dtype)
            g_hi = outs[1][:nh].cpu().numpy()
            k = min(TW_CHECKED, b.n_timelines)
            ok = (np.array_equal(g_tr.view(np.uint8), res.tracks.view(np.uint8)) and np.array_equal(g_hi, res.hit_index)
                  and (nt == info["tracks"] or int(outs[0][nt:nt + 1].cpu().numpy().reshape(-1).view(track_dtype)
                                                   ["timeline"][0]) >= k))
            ent["parity"] = {"timelines": k, "tracks": nt, "hits": nh, "byte_equal": bool(ok)}
            dk = sum(len(tl.t_decay) for tl in b.timelines[:k])
            ent["cpu_baseline"] = {"value": round(dk / osec, 1), "unit": "decays/s", "cores": 1, "kind": "oracle",
                                   "sample": "the first %d timelines (%d decays), one thread, %.1f s" % (k, dk, osec)}
        log("time-sliced leg, %g decays/ns: %s" % (rate, ent))
        out["rates"].append(ent)
        del ts, outs
    return out


def serve_bench(args, finder, log):
    """Served stream: requests of mixed pileup (uniform over 1, 10, 25, 50,
    100 tracks, drawn from a pool of seeded events) arrive as a Poisson
    process at each offered rate and go through the server's continuous
    batching. Latency is the server's completion time minus the request's
    arrival time. A final burst (every request arriving at once, its hit
    arrays gathered from the pool beforehand, as a client would hold them)
    gives the most the served form sustains."""
    import numpy as np
    import torch
    from paper_2511_02742_amd import eventgen
    from paper_2511_02742_amd.hough import HoughServer

    pool = eventgen.mixed_pileup_batch(args.serve_pool, seed0=2_000_000)
    P = len(pool.offsets) - 1
    lens = np.diff(pool.offsets)
    # expected per-event results from one batched call on the pool
    dev = torch.device("cuda", 0)
    out = finder.find(torch.from_numpy(pool.z).to(dev), torch.from_numpy(pool.vane).to(dev),
                      torch.from_numpy(pool.offsets).to(dev))
    cand, whits, info = out.to_host()
    assert info["status"] == 0
    want_nc = np.bincount(cand["event"], minlength=P)
    want_nh = np.bincount(cand["event"], weights=cand["n_hits"], minlength=P).astype(np.int64)
    want_c0 = np.concatenate([[0], np.cumsum(want_nc)])
    want_h0 = np.concatenate([[0], np.cumsum(want_nh)])
    fields = [k for k in cand.dtype.names if k not in ("event", "hit_offset")]

    def mismatches(r, rc, rh):
        """Requests whose candidates (every field but the event number and the
        hit offset, which are request-relative there) or hit lists differ from
        the batched reference's event."""
        ev = idx[r["tag"].astype(np.int64)]
        bad = (r["n_candidates"] != want_nc[ev]) | (r["n_hit_index"] != want_nh[ev])
        ok = ~bad
        nc = r["n_candidates"][ok].astype(np.int64)
        if nc.sum():
            got_i = np.repeat(r["cand_offset"][ok], nc) + (np.arange(nc.sum()) - np.repeat(np.cumsum(nc) - nc, nc))
            want_i = np.repeat(want_c0[ev[ok]], nc) + (np.arange(nc.sum()) - np.repeat(np.cumsum(nc) - nc, nc))
            diff = np.zeros(nc.sum(), bool)
            for k in fields:
                diff |= rc[k][got_i] != cand[k][want_i]
            rel = rc["hit_offset"][got_i] - rc["hit_offset"][np.repeat(r["cand_offset"][ok], nc)]
            wrel = cand["hit_offset"][want_i] - cand["hit_offset"][np.repeat(want_c0[ev[ok]], nc)]
            diff |= rel != wrel
            req = np.repeat(np.nonzero(ok)[0], nc)
            bad[np.unique(req[diff])] = True
        nh = r["n_hit_index"][~bad].astype(np.int64)
        if nh.sum():
            okr = np.nonzero(~bad)[0]
            got_i = np.repeat(r["hit_offset"][okr], nh) + (np.arange(nh.sum()) - np.repeat(np.cumsum(nh) - nh, nh))
            want_i = np.repeat(want_h0[ev[okr]], nh) + (np.arange(nh.sum()) - np.repeat(np.cumsum(nh) - nh, nh))
            diff = rh[got_i] != whits[want_i]
            req = np.repeat(okr, nh)
            bad[np.unique(req[diff])] = True
        return int(bad.sum())

    rates = [float(r) for r in args.serve_rates.split(",") if r] + [float("inf")]
    res = []
    with HoughServer(0, lanes=args.serve_lanes, queue_events=1 << 21, queue_hits=1 << 28) as srv:
        # warm-up
        srv.submit(pool.z, pool.vane, pool.offsets[:65])
        srv.drain(60.0)
        srv.poll_records()
        for rate in rates:
            n = args.serve_events
            rng = np.random.default_rng(12345 + (0 if rate == float("inf") else int(rate)))
            idx = rng.integers(0, P, n)
            chunk = 8192 if rate == float("inf") else 4096

            def gather_chunk(lo, hi):
                sel = idx[lo:hi]
                ln = lens[sel]
                offs = np.zeros(len(sel) + 1, np.int64)
                np.cumsum(ln, out=offs[1:])
                g = np.repeat(pool.offsets[sel] - offs[:-1], ln) + np.arange(offs[-1])
                return pool.z[g], pool.vane[g], offs

            pre = {}
            if rate == float("inf"):
                for lo in range(0, n, chunk):
                    pre[lo] = gather_chunk(lo, min(n, lo + chunk))
            st0 = srv.stats()
            t_start = srv.clock() + 0.1
            arr = t_start + (np.zeros(n) if rate == float("inf") else np.cumsum(rng.exponential(1.0 / rate, n)))
            sub = 0
            recs = []
            got = 0
            mism = 0
            while got < n:
                now = srv.clock()
                while sub < n and arr[sub] - now < 0.2:
                    hi = min(n, sub + chunk)
                    zc, vc, offs = pre.pop(sub) if pre else gather_chunk(sub, hi)
                    acc = srv.submit(zc, vc, offs, tags=np.arange(sub, hi, dtype=np.uint64), t_arrival=arr[sub:hi])
                    assert acc == hi - sub, (acc, hi - sub)
                    sub = hi
                r, rc, rh = srv.poll_records()
                if len(r):
                    recs.append(r)
                    got += len(r)
                    mism += mismatches(r, rc, rh)
                else:
                    time.sleep(0.0002)
            r = np.concatenate(recs)
            st1 = srv.stats()
            assert (r["status"] == 0).all()
            lat = r["t_done"] - r["t_arrival"]
            span = float(r["t_done"].max() - r["t_arrival"].min())
            launches = st1["launches"] - st0["launches"]
            ent = {"offered_per_s": None if rate == float("inf") else rate, "requests": n,
                   "sustained_per_s": round(n / span, 1),
                   "latency_us_p50": round(1e6 * float(np.percentile(lat, 50)), 1),
                   "latency_us_p99": round(1e6 * float(np.percentile(lat, 99)), 1),
                   "queue_us_p50": round(1e6 * float(np.percentile(r["t_admit"] - r["t_arrival"], 50)), 1),
                   "launches": launches, "events_per_launch": round(n / max(launches, 1), 2),
                   "max_lanes_busy": st1["max_lanes_busy"], "mismatches": mism}
            log("served %s: %s" % ("burst" if rate == float("inf") else "%.0f/s" % rate, ent))
            res.append(ent)
        sst = srv.stats()
    return {"workload": "mixed pileup {1,10,25,50,100} tracks + 1%% noise, pool of %d seeded events "
                        "(seeds 2000000..), Poisson arrivals" % P,
            "lanes": args.serve_lanes, "device_arena_bytes": sst["device_bytes"],
            "max_device_bytes_in_use": sst["max_device_bytes_in_use"], "mean_hits": round(float(lens.mean()), 1),
            "admission": "arrived requests, oldest first, while the launch's device block fits the arena's "
                         "largest free block",
            "rates": res}


def refit_bench(args, finder, log):
    """Helix refit of the candidates the finder returns for the uneven batch
    (Poisson(20) tracks per event, seeds 1000000..): gather, initial fit and
    20 Gauss-Newton steps on the GPU (timed with HIP events), the parameter
    error against the float64 oracle on a sample of candidates whose hits all
    come from one generated track, and the momentum resolution against the
    generator truth."""
    import math
    import numpy as np
    import torch
    from paper_2511_02742_amd import eventgen
    from paper_2511_02742_amd.hough import (REFIT_STEPS, momentum_mev, refit_gather, refit_gauss_newton,
                                            refit_init)

    b = eventgen.poisson_batch(args.refit_events)
    dev = torch.device("cuda", 0)
    t = {k: torch.from_numpy(getattr(b, k)).to(dev) for k in ("r", "z", "vane", "offsets")}
    out = finder.find(t["z"], t["vane"], t["offsets"])
    cand, hit_index, info = out.to_host()
    assert info["status"] == 0
    hits = refit_gather(out, t["offsets"], t["r"], t["z"], t["vane"])
    stream = torch.cuda.current_stream(dev)
    times = []
    for rep in range(4):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        p = refit_init(hits).contiguous()
        chi2 = refit_gauss_newton(hits, p)
        e1.record(stream)
        torch.cuda.synchronize(dev)
        if rep > 0:
            times.append(e0.elapsed_time(e1))
    ms = float(np.median(times))
    status = hits.status.cpu().numpy()
    P = p.cpu().numpy().astype(np.float64)
    mom = momentum_mev(p.double()).cpu().numpy()
    n_cand = len(cand)
    # purity and truth momentum of each candidate
    pure = np.zeros(n_cand, bool)
    ptrue = np.zeros(n_cand)
    for c, cd in enumerate(cand):
        ev = b.events[cd["event"]]
        tr = ev.track[hit_index[cd["hit_offset"]:cd["hit_offset"] + cd["n_hits"]]]
        if tr[0] >= 0 and np.all(tr == tr[0]):
            pure[c] = True
            ptrue[c] = ev.p[tr[0]]
    fit = (status == 0)
    sel = fit & pure
    ratio = mom[sel] / ptrue[sel] - 1.0
    res = {"workload": "candidates of %d events, Poisson(20) tracks + 1%% noise (seeds 1000000..)" % args.refit_events,
           "candidates": n_cand, "fitted": int(fit.sum()), "pure_fitted": int(sel.sum()),
           "steps": REFIT_STEPS, "ms": round(ms, 4), "candidates_per_s": round(n_cand / (ms * 1e-3), 1),
           "momentum_bias": round(float(np.median(ratio)), 5),
           "momentum_resolution_68": round(float(np.quantile(np.abs(ratio - np.median(ratio)), 0.68)), 5)}
    if args.refit_oracle > 0 and not args.no_cpu_baseline:
        from oracle.refit_oracle import refit_gn, refit_init as o_init
        floors = np.array([1e-4, 1.0, 1.0, 1.0, 0.01])
        worst = np.zeros(5)
        done = 0
        r_np, z_np, v_np = b.r, b.z, b.vane
        for c in np.nonzero(sel)[0][:args.refit_oracle]:
            cd = cand[c]
            idx = b.offsets[cd["event"]] + hit_index[cd["hit_offset"]:cd["hit_offset"] + cd["n_hits"]]
            p0, s0, a0 = o_init(r_np[idx], z_np[idx], v_np[idx])
            po = refit_gn(p0, r_np[idx], z_np[idx], v_np[idx], s0, a0)
            e = np.abs(P[c] - po) / np.maximum(np.abs(po), floors)
            e[1] = abs(math.remainder(P[c][1] - po[1], 2 * math.pi))
            worst = np.maximum(worst, e)
            done += 1
        res["oracle_sample"] = done
        res["max_param_error_vs_f64"] = {k: float("%.3g" % v) for k, v in
                                         zip(("kappa", "phi0", "d0", "z0", "tan_lambda"), worst)}
    log("refit: %s" % res)
    return res


def _oracle_slice(args):
    """Worker: the oracle over one contiguous slice of events for about
    `seconds` (at least 4 events); returns (events done, seconds)."""
    z, vane, offsets, seconds = args
    from oracle import OracleConfig, oracle_find
    cfg = OracleConfig()
    done = 0
    t0 = time.perf_counter()
    while done < len(offsets) - 1 and (time.perf_counter() - t0 < seconds or done < 4):
        lo, hi = int(offsets[done]), int(offsets[done + 1])
        oracle_find(cfg, z[lo:hi], vane[lo:hi])
        done += 1
    return done, time.perf_counter() - t0


def oracle_all_cores(batch, seconds, log):
    """The same single-thread oracle in independent worker processes (one per
    core of the host's share, at most 16) over disjoint slices of the batch."""
    import multiprocessing as mp
    import numpy as np
    workers = max(1, min(16, os.cpu_count() or 1))
    bounds = np.linspace(0, N_EVENTS, workers + 1).astype(int)
    jobs = []
    for w in range(workers):
        e0, e1 = bounds[w], bounds[w + 1]
        lo, hi = int(batch.offsets[e0]), int(batch.offsets[e1])
        jobs.append((batch.z[lo:hi].copy(), batch.vane[lo:hi].copy(), batch.offsets[e0:e1 + 1] - lo, seconds))
    with mp.get_context("spawn").Pool(workers) as pool:
        res = pool.map(_oracle_slice, jobs)
    done = sum(r[0] for r in res)
    span = max(r[1] for r in res)
    log("cpu oracle, %d processes: %.1f events/s" % (workers, done / span))
    return {"value": round(done / span, 2), "unit": "events/s", "cores": workers, "kind": "oracle",
            "sample": "%d independent single-thread processes over disjoint slices of the same %d pileup-50 "
                      "events, %d events in %.1f s" % (workers, N_EVENTS, done, span)}


def profiled_traffic(name, source):
    """HBM bytes per launch (read + written) from the committed counter
    summary profiles/<name>.txt, or None when it is missing or was taken from
    another version of the kernel source."""
    try:
        from paper_2511_02742_amd.prof_summary import kernel_source_hash
        kv = {}
        with open(os.path.join(ROOT, "profiles", name + ".txt")) as fh:
            for line in fh:
                if ":" in line:
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("kernel_sha256_16") == kernel_source_hash(source) and "fetch_bytes_per_launch" in kv:
            return float(kv["fetch_bytes_per_launch"]) + float(kv["write_bytes_per_launch"])
    except (OSError, ValueError):
        pass
    return None


def _has_run(vanes, length, n_vanes=40):
    """Whether the vane set holds `length` consecutive vanes (cyclic)."""
    return any(all((v + i) % n_vanes in vanes for i in range(length)) for v in vanes)


def eq5_efficiency(batch, cand, hit_index, run=5):
    """Track-finding efficiency of Eq. (5), N_found / N_all: a generated track
    counts as found when one candidate holds its hits on `run` consecutive
    vanes. Returned over all generated tracks and over the tracks whose own
    hits span such a run (the ones a seed can find at all)."""
    import numpy as np
    found = set()
    for cd in cand:
        ev = batch.events[cd["event"]]
        idx = hit_index[cd["hit_offset"]:cd["hit_offset"] + cd["n_hits"]]
        tr, vn = ev.track[idx], ev.vane[idx]
        for t in np.unique(tr[tr >= 0]):
            if _has_run(set(vn[tr == t].tolist()), run):
                found.add((int(cd["event"]), int(t)))
    n_all = n_findable = n_found_findable = 0
    for e, ev in enumerate(batch.events):
        n_all += ev.n_tracks
        for t in np.unique(ev.track[ev.track >= 0]):
            if _has_run(set(ev.vane[ev.track == t].tolist()), run):
                n_findable += 1
                n_found_findable += (e, int(t)) in found
    return {"found": len(found), "all_tracks": n_all, "findable_tracks": n_findable,
            "efficiency": round(len(found) / max(n_all, 1), 4),
            "efficiency_findable": round(n_found_findable / max(n_findable, 1), 4)}


def seeded_fraction(batch, cand, hit_index, min_hits):
    """Share of the generated tracks with at least min_hits hits that some
    candidate seeds: at least min_hits of the candidate's hits, and more than
    half of them, come from that track."""
    import numpy as np
    seeded = set()
    for cd in cand:
        ev = batch.events[cd["event"]]
        tr = ev.track[hit_index[cd["hit_offset"]:cd["hit_offset"] + cd["n_hits"]]]
        tr = tr[tr >= 0]
        if len(tr) == 0:
            continue
        t, k = np.unique(tr, return_counts=True)
        i = int(np.argmax(k))
        if k[i] >= min_hits and 2 * k[i] > cd["n_hits"]:
            seeded.add((int(cd["event"]), int(t[i])))
    findable = 0
    hit = 0
    for e, ev in enumerate(batch.events):
        t, k = np.unique(ev.track[ev.track >= 0], return_counts=True)
        for tt in t[k >= min_hits]:
            findable += 1
            hit += (e, int(tt)) in seeded
    return hit / max(findable, 1), findable


def coarse_fine_bench(args, batch, z, vane, offs, log, lds_vote_peak=None, refs=None):
    """The paper's two-stage histogram (18 x 100 coarse, 10 x 10 fine, on the
    180 x 1000 grid) on the same pileup-50 batch, against full-grid argmax and
    nms on the same grid: events/s, finder kernel time, Eq. (4) evaluations,
    candidates and the share of findable generated tracks each one seeds."""
    import numpy as np
    import torch
    from paper_2511_02742_amd.hough import HoughFinder
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream(dev)
    res = {"workload": "the same %d pileup-50 events, 180 x 1000 grid, T=6, a=0" % N_EVENTS}
    for name, kw in (("coarse_fine", {"peak_mode": 2}), ("argmax", {"peak_mode": 0}), ("nms", {"peak_mode": 1})):
        f = HoughFinder(0, n_theta=180, n_rho=1000, **kw)
        out = f.alloc_outputs(N_EVENTS, batch.n_hits)
        for _ in range(args.warmup):
            f.find(z, vane, offs, out=out, stream=stream)
        torch.cuda.synchronize(dev)
        f.set_timing(True)
        f.timing(reset=True)
        t1 = time.perf_counter()
        for _ in range(args.steps):
            f.find(z, vane, offs, out=out, stream=stream)
        torch.cuda.synchronize(dev)
        wall = time.perf_counter() - t1
        f.set_timing(False)
        kern_ms, launches = f.timing(reset=True)
        cand, hits, info = out.to_host()
        assert info["status"] == 0, info
        frac, findable = seeded_fraction(batch, cand, hits, 6)
        e5 = eq5_efficiency(batch, cand, hits)
        kavg = kern_ms / max(launches, 1)
        res[name] = {"events_per_s": round(N_EVENTS * args.steps / wall, 1),
                     "ms_per_step": round(1e3 * wall / args.steps, 4), "kernel_avg_ms": round(kavg, 4),
                     "kernel": "k_find_cf" if name == "coarse_fine" else "k_find",
                     "evals": info["evals"], "evals_per_s": round(info["evals"] / (kavg * 1e-3), 1),
                     "votes": info["votes"],
                     "lds_frac_vote_pattern": round(info["votes"] / (kavg * 1e-3) / lds_vote_peak, 4)
                     if lds_vote_peak else None,
                     "candidates": info["candidates"], "iters": info["iters"],
                     "seeded_track_fraction": round(frac, 4),
                     "efficiency_eq5": e5["efficiency"], "efficiency_eq5_findable": e5["efficiency_findable"],
                     "ordered": info["ordered"],
                     "parity": parity_record(cand, hits, refs["cf_" + name], N_EVENTS)
                     if refs and ("cf_" + name) in refs else None}
        res["findable_tracks"] = findable
        log("coarse-fine leg, %s: %s" % (name, res[name]))
    cf = res["coarse_fine"]
    flops = FLOPS_PER_VOTE * cf["evals"]
    achieved = flops / (cf["kernel_avg_ms"] * 1e-3) / 1e12
    cf["roofline"] = {"bound": "alu", "achieved": round(achieved, 4), "peak": round(VALU_PEAK_TFLOPS, 2),
                      "unit": "TFLOP/s", "frac": round(achieved / VALU_PEAK_TFLOPS, 4),
                      "traffic": profiled_traffic("k_find_cf_pileup50", "hough_cf.hip")}
    return res


if __name__ == "__main__":
    main()
